// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rbffd.h"

struct rbffd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  int n_cu = 256;
  void *scratch = nullptr;  // this device's scratch of rbffd_weights_noalloc
  int wshape[RBFFD_WEIGHT_BUCKETS] = {};  // weights launch shape per size bucket (rbffd_weights_tune)
};

// Error helper: records a message and returns the code.
int rbffd_fail(rbffd_ctx *ctx, int code, const char *fmt, ...);

#define RBFFD_HIP(ctx, call)                                                         \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return rbffd_fail((ctx), RBFFD_EDEVICE, "%s failed: %s (%s:%d)", #call,        \
                        hipGetErrorString(e_), __FILE__, __LINE__);                  \
  } while (0)

// A workspace request: a failed allocation is ENOMEM; a request beyond a
// fixed region (which the callers' size checks rule out) is reported as such.
#define RBFFD_WS(ctx, ws, call)                                                                   \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return rbffd_fail((ctx), (ws).fixed() ? RBFFD_EINVAL : RBFFD_ENOMEM,                        \
                        (ws).fixed() ? "scratch region exhausted (%s:%d)" : "device allocation "  \
                                                                            "failed (%s:%d)",     \
                        __FILE__, __LINE__);                                                      \
  } while (0)

// Entry into a library call: select the context's device and drop a stale
// "last error" that an unrelated earlier call on this thread may have left
// (the not-ready status of an event or stream query, for instance), so the
// launch checks after our own launches report those launches only. A device
// fault is not lost: it stays with the context and fails later calls.
#define RBFFD_ENTER(ctx)                                  \
  do {                                                    \
    RBFFD_HIP((ctx), hipSetDevice((ctx)->device));        \
    (void)hipGetLastError();                              \
  } while (0)

// Scoped device buffer (stream-ordered free is not needed: buffers live
// until the owning call or object ends, after a synchronisation).
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  hipError_t alloc(size_t n) {
    release();
    bytes = n;
    return n ? hipMalloc(&p, n) : hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// Device scratch of one search or weights call. Without a region every
// request is a hipMalloc, released when the call ends; with a fixed region
// requests are carved from it in order, 256-byte aligned, and a request
// beyond its end fails without allocating.
class Workspace {
 public:
  Workspace() = default;
  Workspace(void *region, size_t cap) : base_(static_cast<char *>(region)), cap_(cap) {}
  Workspace(const Workspace &) = delete;
  Workspace &operator=(const Workspace &) = delete;
  ~Workspace() {
    for (void *p : owned_) (void)hipFree(p);
  }
  bool fixed() const { return base_ != nullptr; }
  size_t used() const { return used_; }
  // `bytes` of device memory in *out (null for zero bytes)
  hipError_t get(size_t bytes, void **out) {
    *out = nullptr;
    if (bytes == 0) return hipSuccess;
    if (base_) {
      const size_t at = (used_ + 255) & ~size_t(255);
      if (at > cap_ || bytes > cap_ - at) return hipErrorOutOfMemory;
      *out = base_ + at;
      used_ = at + bytes;
      return hipSuccess;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) owned_.push_back(p);
    *out = p;
    used_ += bytes;
    return e;
  }
  template <class T> hipError_t get(size_t count, T **out) {
    void *p = nullptr;
    hipError_t e = get(count * sizeof(T), &p);
    *out = static_cast<T *>(p);
    return e;
  }

 private:
  char *base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  std::vector<void *> owned_;
};

// Device scratch of the search for n nodes and nc centres, of the argument
// checks, and of the weights (after the search) for nc centres, as the
// Workspace requests them (each rounded up to 256 bytes): the size a fixed
// region needs. The constants are the search's box blocks and scan tile and
// the weights' count array.
constexpr int KNN_BOX_BLOCKS = 512;
constexpr int KNN_SCAN_TILE = 4096;
constexpr int WEIGHTS_COUNTS = 40;
constexpr size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t knn_scratch_bytes(int64_t n_nodes, int64_t n_centers) {
  // box partials, box + overflow count, cell counts, cell starts, scan tile
  // sums, nodes by cell, centres left to the dense-cluster kernel
  const size_t n = static_cast<size_t>(n_nodes), cells = n + 16;
  const size_t tiles = (cells + KNN_SCAN_TILE - 1) / KNN_SCAN_TILE;
  const size_t nc = static_cast<size_t>(n_centers > 1 ? n_centers : 1);
  return round256(sizeof(double) * 4 * KNN_BOX_BLOCKS) + round256(sizeof(double) * 8) +
         round256(sizeof(int) * cells) + round256(sizeof(int) * (cells + 1)) + round256(sizeof(int) * tiles) +
         round256(sizeof(int) * n) + round256(sizeof(int) * nc);
}
constexpr size_t CHECK_SCRATCH_BYTES = 256;
constexpr size_t weights_scratch_bytes(int64_t n_centers) {
  // counts and queues, bucket lists, status (when the caller passes none),
  // stencils left by the two-systems-per-wavefront kernel,
  // FP32-factorisation stencils to solve again
  const size_t nc = static_cast<size_t>(n_centers > 1 ? n_centers : 1);
  return round256(WEIGHTS_COUNTS * sizeof(int)) + round256(nc * sizeof(int)) + round256(nc * sizeof(int32_t)) +
         round256(nc * sizeof(int)) + round256(nc * sizeof(int));
}

// ---- argument checks on the device (check.hip) ----
// Every per-stencil parameter and index of a search (`weights` false) or a
// weights call is checked before anything is written: centre indices, n, and
// for weights m, l, n >= M(l), n + M <= 128, Laplacian^k continuity and the
// given stencils' indices. Synchronises; RBFFD_EINVAL names the first bad
// stencil.
int check_stencils_device(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops, bool weights,
                          Workspace &ws);

// ---- stencil search (knn.hip) ----
int knn_run(rbffd_ctx *ctx, const rbffd_stencils *st, int32_t *idx, Workspace &ws);

// ---- weights (weights.hip) ----
// `shapes`: launch shape per size bucket (NULL: the context's tuned ones);
// `bucket_ev`: NULL, or two events per bucket recorded around its launches.
int weights_run(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops,
                int precision, const int32_t *idx, double *w, int32_t *status, int32_t *n_bad,
                Workspace &ws, const int *shapes = nullptr, hipEvent_t *bucket_ev = nullptr);
int weights_tune(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops, int precision,
                 const int32_t *idx, double *w, int32_t *status, int32_t *n_bad, int32_t *shapes, double *ms);
int weights_shape_count(int bucket);

// ---- right-hand side model (model.hip / rhs.hip) ----
struct StageArgs;
int model_create_impl(rbffd_ctx *ctx, const rbffd_model_desc *d, rbffd_model **out);
int model_destroy_impl(rbffd_model *m);
int model_ghost(rbffd_ctx *ctx, rbffd_model *m, void *state);
int model_rhs(rbffd_ctx *ctx, rbffd_model *m, double t, void *state, void *tendency);
int model_step(rbffd_ctx *ctx, rbffd_model *m, void *state, double *t, double dt,
               int64_t n_steps, int tableau);
int64_t model_bytes_per_node(rbffd_model *m);
int model_profile(rbffd_model *m, int enable);
int model_profile_read(rbffd_model *m, double *total_ms, int64_t *launches);
int stream_copy(rbffd_ctx *ctx, void *dst, const void *src, int64_t bytes);
int model_tune(rbffd_ctx *ctx, rbffd_model *m, void *state, int *chosen, double *best_us);
int mfma_probe(rbffd_ctx *ctx, int shape, float *out, int64_t n_out, int iters, int64_t *flops);
int closure_create(rbffd_ctx *ctx, rbffd_model *m, const rbffd_closure_desc *d, rbffd_closure **out);
int closure_destroy(rbffd_closure *cl);
float *closure_params(rbffd_closure *cl);
int closure_forward(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, float *out);
int closure_tune(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, int *chosen, double *best_us);
int closure_gradient(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, const float *target, float *grad,
                     double *loss);
int closure_train_step(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, const float *target, double lr,
                       double *loss);
int closure_step(rbffd_ctx *ctx, rbffd_closure *cl, void *state, double *t, double dt, int64_t n_steps, int tableau,
                 int64_t *n_fallback);

// Launch geometry helper: grid of blocks covering n items.
inline unsigned grid_for(int64_t n, int block) {
  return static_cast<unsigned>((n + block - 1) / block);
}

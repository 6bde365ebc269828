// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

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

// ---- stencil search (knn.hip) ----
int knn_run(rbffd_ctx *ctx, const rbffd_stencils *st, int32_t *idx);

// ---- weights (weights.hip) ----
int weights_run(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops,
                int precision, const int32_t *idx, double *w, int32_t *status, int32_t *n_bad);

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

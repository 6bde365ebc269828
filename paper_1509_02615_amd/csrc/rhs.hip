// B1-B4: ghost closure, fused gather-stencil right-hand side, RK stages.
//
// The right-hand side is a memory-bound ELL product: for every node i and
// slot k the kernel streams the slot-major record (index + weights of
// every operator) once, coalesced across the wavefront, gathers the
// neighbour's fields (all four fields of a node are one 16- or 32-byte
// vector, so a gather is one load) and accumulates every derivative the
// equations need. The pointwise physics and the Runge-Kutta stage update are
// fused into the epilogue, so one launch per stage reads each stream once.
//
// Navier-Stokes (Eqs. uEq, wEq, thetaEq, piEq): 15 dot products per node --
// Dx and Dz of u, w, theta', pi'; Lap of u, w, theta' (mu Lap); Lap^k of all
// four (hyperviscosity, Section 5.3). Transport (Section 6.1, flux form):
// the velocity shape is folded into one weight per slot, 2 dot products.
//
// Reduced precision: FP32 fields use centre-subtracted sums
// sum_k w_k (f_j - f_i), which equal sum_k w_k f_j because derivative
// weights sum to zero (they reproduce constants, Section 3). Two kinds of sum
// run in FP64 on weights corrected towards their FP64 values: the
// hyperviscosity sums (they cancel strongly), and the divergence u_x + w_z,
// whose term in the pressure equation (Eq. piEq) nearly cancels w dpi-bar/dz
// in a developed flow, so that its FP32 rounding would dominate the pressure
// tendency's error.
//
// Launch geometry: 256-thread blocks, thread = (node, member); block ids are
// remapped so that each of the 8 XCDs (which take block ids round-robin)
// works on one contiguous node range and its L2 sees neighbouring gathers.
#include <hip/hip_ext.h>

#include <algorithm>
#include <climits>
#include <type_traits>
#include <cmath>

#include "model.hpp"

namespace {

constexpr int RHS_BLOCK = 256;  // closure and transport kernels

// Launch shapes of the Navier-Stokes stage kernel: block size, slot
// unrolling and whether the weight stream is loaded non-temporally (each
// launch reads it exactly once; keeping it out of the caches leaves them to
// the neighbour gathers). rbffd_model_tune times them on the model's data.
// Defaults, measured on the 524,288-node channel: shape 0 for FP32 and BF16
// records, shape 2 for FP64.
struct Shape {
  int block, unroll;
  bool nt;
};
constexpr Shape kShapes[] = {{256, 1, true}, {256, 2, false}, {512, 2, false},
                             {128, 1, true}, {512, 1, true},  {256, 4, true}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
inline int default_shape(int wdt) { return wdt == RBFFD_F64 ? 2 : 0; }
template <int S> struct StageShape {
  static constexpr int block = kShapes[S].block, unroll = kShapes[S].unroll;
  static constexpr bool nt = kShapes[S].nt;
};

typedef float nat_f4 __attribute__((ext_vector_type(4)));
typedef double nat_d2 __attribute__((ext_vector_type(2)));
template <bool NT, class T> __device__ __forceinline__ T stream_load(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT> __device__ __forceinline__ float4 stream_load4(const float4 *p) {
  if constexpr (NT) {
    nat_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nat_f4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  }
  return *p;
}
template <bool NT> __device__ __forceinline__ double2 stream_load2(const double2 *p) {
  if constexpr (NT) {
    nat_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nat_d2 *>(p));
    return make_double2(v.x, v.y);
  }
  return *p;
}
template <bool NT> __device__ __forceinline__ uint2 stream_load2u(const uint2 *p) {
  if constexpr (NT) {
    const unsigned *q = reinterpret_cast<const unsigned *>(p);
    return make_uint2(__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1));
  }
  return *p;
}
template <bool NT> __device__ __forceinline__ uint3 stream_load3(const uint3 *p) {
  if constexpr (NT) {
    const unsigned *q = reinterpret_cast<const unsigned *>(p);
    return make_uint3(__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1),
                      __builtin_nontemporal_load(q + 2));
  }
  return *p;
}

// Neighbour offset s. With a wave-uniform s (one node per wavefront) the
// aligned dword holding it is loaded, so the load can go through the scalar
// cache (scalar loads are dword-sized) instead of a vector load whose
// latency would precede every gather address.
template <bool NT, bool UNIFORM> __device__ __forceinline__ int load_off(const int16_t *off16, int64_t s) {
  if constexpr (UNIFORM) {
    const unsigned wd = reinterpret_cast<const unsigned *>(off16)[s >> 1];
    return static_cast<int16_t>(wd >> (16 * static_cast<int>(s & 1)));
  }
  return stream_load<NT>(off16 + s);
}

template <int BLOCK = RHS_BLOCK> __device__ __forceinline__ int64_t xcd_thread() {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  const int64_t full = (nb / 8) * 8;
  const int64_t lb = b >= full ? b : (b % 8) * (nb / 8) + b / 8;
  return lb * BLOCK + threadIdx.x;
}

__device__ __forceinline__ int64_t xcd_block() {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  const int64_t full = (nb / 8) * 8;
  if (b >= full) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

template <class FT> struct F4 {
  FT v[4];
};

__device__ __forceinline__ F4<float> load4(const float *p) {
  float4 q = *reinterpret_cast<const float4 *>(p);
  return F4<float>{{q.x, q.y, q.z, q.w}};
}
__device__ __forceinline__ F4<double> load4(const double *p) {
  double2 a = reinterpret_cast<const double2 *>(p)[0];
  double2 b = reinterpret_cast<const double2 *>(p)[1];
  return F4<double>{{a.x, a.y, b.x, b.y}};
}
__device__ __forceinline__ void store4(float *p, const double *v) {
  *reinterpret_cast<float4 *>(p) = make_float4(static_cast<float>(v[0]), static_cast<float>(v[1]),
                                               static_cast<float>(v[2]), static_cast<float>(v[3]));
}
__device__ __forceinline__ void store4(double *p, const double *v) {
  reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
}
// v - fl32(v) for each of four FP64 values, as FP32 (exact to about 2^-48 of v)
__device__ __forceinline__ void store_remainder(float *p, const double *v) {
  float r[4];
  for (int c = 0; c < 4; ++c) r[c] = static_cast<float>(v[c] - static_cast<double>(static_cast<float>(v[c])));
  *reinterpret_cast<float4 *>(p) = make_float4(r[0], r[1], r[2], r[3]);
}

__device__ __forceinline__ float bf16f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

struct NSArgs {
  const void *ys;     // fields the derivatives are taken of  [N][E][4]
  const void *yn;     // base of the stage update (y_n)
  void *out;          // tendency or next stage
  void *acc;          // RK4 accumulator
  const int *idx_t;      // full neighbour indices (read for OFF_FAR offsets only)
  const int16_t *off16;  // neighbour offsets j - i (F64 records)
  const uint32_t *aux32; // neighbour offset and weight corrections (FP32 records)
  const void *rec;
  const void *rec2;      // second record stream (BF16 layout)
  const uint8_t *kind;
  const double *pibar;
  const int *order;   // member-wavefront mode: node of each wavefront-sized unit (or NULL)
  const void *rec_t;  // with `order`, FP32 ensemble records in that order (or NULL)
  const float *ghrem; // FP32 fields: each ghost value's FP64 remainder past its FP32
                      // rounding in the state, [N - Na][E][4] (or NULL)
  int64_t Na;
  int n, E;
  double c_p, rcv, g, theta_bar, mu, hv, dpibar, u_bar;
  double ca, cb;
  int mode;      // 0: out = f; 1: out = yn + ca f; 2: out = acc + ca f
  int acc_mode;  // 0: none; 1: acc = yn + cb f; 2: acc += cb f
  DevMisc *misc;
  int check;     // record the step of the first non-finite output
};

// MW ("member wavefront"): the ensemble size is a multiple of 64, so a
// wavefront holds 64 members of one node; the node index is then
// wave-uniform and the weight records are fetched once per wavefront through
// the scalar cache and broadcast (the gathers stay vector loads, 64
// consecutive members = one contiguous 1 KiB span in FP32).
template <class FT, int WDT, int S, bool MW = false>
__global__ __launch_bounds__(StageShape<S>::block) void ns_stage_kernel(NSArgs a) {
  using SH = StageShape<S>;
  constexpr bool NT = SH::nt && !MW;
  const int64_t t = xcd_thread<SH::block>();
  if (t >= a.Na * a.E) return;
  const int E = a.E;
  int64_t i = E == 1 ? t : t / E;
  const int e = static_cast<int>(t - i * E);  // the member
  int64_t ri = i;  // column of the node's records: the node, or its place in the traversal
  if constexpr (MW) {  // a wave-uniform node, taken in the model's traversal order
    const int li = __builtin_amdgcn_readfirstlane(static_cast<int>(i));
    i = a.order ? a.order[li] : li;
    ri = a.rec_t ? li : i;
  }
  const FT *ys = static_cast<const FT *>(a.ys);
  const F4<FT> own = load4(ys + (i * E + e) * 4);
  const int n = a.n;
  const int64_t Na = a.Na;
  // the 15 stencil sums, in FP64 for the epilogue: Dx and Dz of the four
  // fields, Lap of u, w, theta', Lap^k of all four; ux and wz the divergence
  double gx[4], gz[4], gl[3], shv[4] = {0.0, 0.0, 0.0, 0.0}, ux, wz;
  if constexpr (WDT == RBFFD_F32 && MW) {
    // FP32 ensembles of a multiple of 64 members: the FP64 record (RecMW) is
    // wave-uniform, and every sum is taken in FP64 from exact differences.
    // The vector unit issues an FP64 multiply-add at the rate of an FP32 one
    // (packed FP32 is not used), so FP64 sums cost no more and spare the
    // per-slot conversions of FP64 weights to FP32
    const double o[4] = {own.v[0], own.v[1], own.v[2], own.v[3]};
    double sx[4] = {0.0, 0.0, 0.0, 0.0}, sz[4] = {0.0, 0.0, 0.0, 0.0}, sl[3] = {0.0, 0.0, 0.0};
    const RecMW *recs = static_cast<const RecMW *>(a.rec_t ? a.rec_t : a.rec) + ri;
    // the neighbour's member vector: a wave-uniform base (scalar arithmetic)
    // plus the lane's 16-byte offset
    auto gather = [&](int j) { return load4(ys + static_cast<int64_t>(j) * (4 * E) + 4 * static_cast<uint32_t>(e)); };
    if (a.ghrem && (a.kind[i] & KIND_REACH)) {
      // a node next to a wall (wave-uniform): the ghost neighbours' closure
      // values' FP64 remainders are added as well, as in the one-member path
#pragma unroll 1
      for (int k = 0; k < n; ++k) {
        const RecMW r = recs[k * Na];
        if (r.idx < Na) continue;
        const float4 q4 = *reinterpret_cast<const float4 *>(a.ghrem + ((r.idx - Na) * E + e) * 4);
        const float q[4] = {q4.x, q4.y, q4.z, q4.w};
        const double wl = r.lap;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double d = q[c];
          sx[c] = fma(r.dx, d, sx[c]);
          sz[c] = fma(r.dz, d, sz[c]);
          if (c < 3) sl[c] = fma(wl, d, sl[c]);
          shv[c] = fma(r.hv, d, shv[c]);
        }
      }
    }
#pragma unroll SH::unroll
    for (int k = 0; k < n; ++k) {
      const RecMW r = recs[k * Na];
      const F4<FT> f = gather(r.idx);
      const double wl = r.lap;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double d = static_cast<double>(f.v[c]) - o[c];
        sx[c] = fma(r.dx, d, sx[c]);
        sz[c] = fma(r.dz, d, sz[c]);
        if (c < 3) sl[c] = fma(wl, d, sl[c]);
        shv[c] = fma(r.hv, d, shv[c]);
      }
    }
    for (int c = 0; c < 4; ++c) {
      gx[c] = sx[c];
      gz[c] = sz[c];
      if (c < 3) gl[c] = sl[c];
    }
    ux = sx[0];
    wz = sz[1];
  } else {
    FT sdx[4] = {0, 0, 0, 0}, sdz[4] = {0, 0, 0, 0}, slp[3] = {0, 0, 0};
    // reduced-precision layouts: the divergence u_x + w_z in FP64, from exact
    // differences and weights corrected towards FP64 (FP64 layout: sdx[0], sdz[1])
    double sux = 0.0, swz = 0.0;
    constexpr bool DIV64 = WDT != RBFFD_F64;
    const double own_u = static_cast<double>(own.v[0]), own_w = static_cast<double>(own.v[1]);
    // slot k's neighbour and weights (the weights corrected towards FP64
    // for the FP64 sums)
    struct Slot {
      int j;
      FT wdx, wdz, wlp;
      double whv, wdx64, wdz64;
    };
    auto slot = [&](int k) {
      const int64_t s = static_cast<int64_t>(k) * Na + i;
      Slot q{};
      int off;
      if constexpr (WDT == RBFFD_F64) {
        const double2 r0 = stream_load2<NT>(reinterpret_cast<const double2 *>(a.rec) + 2 * s);
        const double2 r1 = stream_load2<NT>(reinterpret_cast<const double2 *>(a.rec) + 2 * s + 1);
        off = load_off<NT, MW>(a.off16, s);
        q.wdx = r0.x;
        q.wdz = r0.y;
        q.wlp = r1.x;
        q.whv = r1.y;
      } else if constexpr (WDT == RBFFD_F32) {
        const float4 r = stream_load4<NT>(reinterpret_cast<const float4 *>(a.rec) + s);
        const uint32_t x = stream_load<NT>(a.aux32 + s);
        off = static_cast<int16_t>(x >> 16);
        q.wdx = r.x;
        q.wdz = r.y;
        q.wlp = r.z;
        // corrections: bits 15-10 (Lap^k), 9-5 (Dx), 4-0 (Dz), signed
        const int qh = static_cast<int>(x << 16) >> 26, qx = static_cast<int>(x << 22) >> 27,
                  qz = static_cast<int>(x << 27) >> 27;
        const double hh = r.w, hx = r.x, hz = r.y;
        q.whv = fma(hh, static_cast<double>(qh) * HV_Q_SCALE, hh);
        q.wdx64 = fma(hx, static_cast<double>(qx) * D_Q_SCALE, hx);
        q.wdz64 = fma(hz, static_cast<double>(qz) * D_Q_SCALE, hz);
      } else {
        const uint2 r = stream_load2u<NT>(reinterpret_cast<const uint2 *>(a.rec) + s);
        const uint2 x = stream_load2u<NT>(reinterpret_cast<const uint2 *>(a.rec2) + s);
        // RecBF16X: {float hv, int8 hvq, lapq, dxq, dzq}
        const float bx = __uint_as_float(r.x << 16), bz = __uint_as_float(r.x & 0xffff0000u);
        const float bl = __uint_as_float(r.y << 16);
        q.wdx = fmaf(bx, static_cast<float>(static_cast<int>(x.y << 8) >> 24) * BF_Q_SCALE, bx);
        q.wdz = fmaf(bz, static_cast<float>(static_cast<int>(x.y) >> 24) * BF_Q_SCALE, bz);
        q.wlp = fmaf(bl, static_cast<float>(static_cast<int>(x.y << 16) >> 24) * BF_Q_SCALE, bl);
        off = static_cast<int16_t>(r.y >> 16);
        const double hh = __uint_as_float(x.x);
        q.whv = fma(hh, static_cast<double>(static_cast<int>(x.y << 24) >> 24) * HV_Q8_SCALE, hh);
        q.wdx64 = q.wdx;
        q.wdz64 = q.wdz;
      }
      if (__builtin_expect(off == OFF_FAR, 0))
        q.j = a.idx_t[s];  // a neighbour beyond +-32767 (a ghost of the first rows)
      else
        q.j = static_cast<int>(i) + off;
      return q;
    };
    // one slot's sums; `ghosts`: the model keeps its ghost values' FP64
    // remainders (FP32 fields), and a ghost neighbour adds its remainder
    // into every sum: the FP32 state holds the closure value rounded, and
    // next to a wall that rounding is a large part of the stencil
    // differences (which the Lap^k weights amplify)
    auto step = [&](const Slot &q, auto ghosts) {
      const F4<FT> f = load4(ys + (static_cast<int64_t>(q.j) * E + e) * 4);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const FT d = f.v[c] - own.v[c];
        if (!DIV64 || c != 0) sdx[c] = fma(q.wdx, d, sdx[c]);
        if (!DIV64 || c != 1) sdz[c] = fma(q.wdz, d, sdz[c]);
        if (c < 3) slp[c] = fma(q.wlp, d, slp[c]);
        shv[c] = fma(q.whv, static_cast<double>(d), shv[c]);
      }
      if constexpr (DIV64) {
        sux = fma(q.wdx64, static_cast<double>(f.v[0]) - own_u, sux);
        swz = fma(q.wdz64, static_cast<double>(f.v[1]) - own_w, swz);
      }
      if constexpr (decltype(ghosts)::value && std::is_same<FT, float>::value) {
        if (q.j >= Na) {
          const float4 r4 = *reinterpret_cast<const float4 *>(a.ghrem + ((q.j - Na) * E + e) * 4);
          const float r[4] = {r4.x, r4.y, r4.z, r4.w};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (!DIV64 || c != 0) sdx[c] = fma(q.wdx, r[c], sdx[c]);
            if (!DIV64 || c != 1) sdz[c] = fma(q.wdz, r[c], sdz[c]);
            if (c < 3) slp[c] = fma(q.wlp, r[c], slp[c]);
            shv[c] = fma(q.whv, static_cast<double>(r[c]), shv[c]);
          }
          if constexpr (DIV64) {
            sux = fma(q.wdx64, static_cast<double>(r[0]), sux);
            swz = fma(q.wdz64, static_cast<double>(r[1]), swz);
          }
        }
      }
    };
    if (a.ghrem) {
#pragma unroll SH::unroll
      for (int k = 0; k < n; ++k) step(slot(k), std::true_type{});
    } else {
#pragma unroll SH::unroll
      for (int k = 0; k < n; ++k) step(slot(k), std::false_type{});
    }
    for (int c = 0; c < 4; ++c) {
      gx[c] = static_cast<double>(sdx[c]);
      gz[c] = static_cast<double>(sdz[c]);
      if (c < 3) gl[c] = static_cast<double>(slp[c]);
    }
    ux = DIV64 ? sux : gx[0];
    wz = DIV64 ? swz : gz[1];
  }
  // Eqs. uEq..piEq (perturbation form), evaluated in FP64; a uniform
  // background wind u_bar joins u in the advective terms
  const double u = own.v[0], w = own.v[1], th = own.v[2], pi = own.v[3];
  const double ua = u + a.u_bar;
  const double cp_th = a.c_p * (a.theta_bar + th);
  double f[4];
  f[0] = -ua * ux - w * gz[0] - cp_th * gx[3] + a.mu * gl[0] + a.hv * shv[0];
  f[1] = -ua * gx[1] - w * wz - cp_th * gz[3] + a.g * th / a.theta_bar + a.mu * gl[1] + a.hv * shv[1];
  f[2] = -ua * gx[2] - w * gz[2] + a.mu * gl[2] + a.hv * shv[2];
  f[3] = -ua * gx[3] - w * (a.dpibar + gz[3]) - a.rcv * (a.pibar[i] + pi) * (ux + wz) + a.hv * shv[3];
  const uint8_t kd = a.kind[i];
  if (kd & KIND_ZWALL) f[1] = 0.0;  // w stays 0 on walls normal to z
  if (kd & KIND_XWALL) f[0] = 0.0;  // u stays 0 on walls normal to x
  const int64_t o = (i * E + e) * 4;
  double r[4];
  if (a.mode == 0) {
    for (int c = 0; c < 4; ++c) r[c] = f[c];
  } else {
    const F4<FT> b = load4(static_cast<const FT *>(a.mode == 1 ? a.yn : a.acc) + o);
    for (int c = 0; c < 4; ++c) r[c] = static_cast<double>(b.v[c]) + a.ca * f[c];
    if (a.acc_mode) {
      const F4<FT> base = load4(static_cast<const FT *>(a.acc_mode == 1 ? a.yn : a.acc) + o);
      double q[4];
      for (int c = 0; c < 4; ++c) q[c] = static_cast<double>(base.v[c]) + a.cb * f[c];
      store4(static_cast<FT *>(a.acc) + o, q);
    }
  }
  store4(static_cast<FT *>(a.out) + o, r);
  if (a.check) {
    bool fin = isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]) && isfinite(r[3]);
    if (!fin) atomicMin(&a.misc->nonfinite_step, a.misc->step_ctr);
  }
}

struct AdvArgs {
  const void *ys, *yn;
  void *out, *acc;
  const int *idx_t;
  const RecAdv *rec;
  int64_t Na;
  int n, E;
  double hv, omega;     // velocity factor cos(omega * t)
  double t_fixed;       // stage time when misc == nullptr
  double t_off, dt;     // stage time = t0 + step_ctr * dt + t_off
  double ca, cb;
  int mode, acc_mode;
  DevMisc *misc;
  int check;
  const int *mir_off, *mir_list;  // stage updates: also write each node's mirror ghosts (or null)
};

template <class FT>
__global__ __launch_bounds__(RHS_BLOCK) void adv_stage_kernel(AdvArgs a) {
  const int64_t t = xcd_block() * RHS_BLOCK + threadIdx.x;
  if (t >= a.Na * a.E) return;
  const int E = a.E;
  const int64_t i = E == 1 ? t : t / E;
  const int e = static_cast<int>(t - i * E);
  const FT *ys = static_cast<const FT *>(a.ys);
  double sa = 0.0, sh = 0.0;
  const int64_t Na = a.Na;
#pragma unroll 4
  for (int k = 0; k < a.n; ++k) {
    const int64_t s = static_cast<int64_t>(k) * Na + i;
    const int j = a.idx_t[s];
    const RecAdv r = a.rec[s];
    const double v = ys[static_cast<int64_t>(j) * E + e];
    sa = fma(r.adv, v, sa);
    sh = fma(r.hv, v, sh);
  }
  double ts = a.t_fixed;
  if (a.misc) ts = (a.misc->t0 + static_cast<double>(a.misc->step_ctr) * a.dt) + a.t_off;
  const double f = -cos(a.omega * ts) * sa + a.hv * sh;
  const int64_t o = i * E + e;
  double r;
  if (a.mode == 0) {
    r = f;
  } else {
    const FT *b = static_cast<const FT *>(a.mode == 1 ? a.yn : a.acc);
    r = static_cast<double>(b[o]) + a.ca * f;
    if (a.acc_mode) {
      const FT *base = static_cast<const FT *>(a.acc_mode == 1 ? a.yn : a.acc);
      static_cast<FT *>(a.acc)[o] = static_cast<FT>(static_cast<double>(base[o]) + a.cb * f);
    }
  }
  static_cast<FT *>(a.out)[o] = static_cast<FT>(r);
  if (a.mir_off) {  // the value the mirror boundary would copy into this node's ghosts
    for (int g = a.mir_off[i]; g < a.mir_off[i + 1]; ++g)
      static_cast<FT *>(a.out)[(Na + a.mir_list[g]) * E + e] = static_cast<FT>(r);
  }
  if (a.check && !isfinite(r)) atomicMin(&a.misc->nonfinite_step, a.misc->step_ctr);
}

struct GArgs {
  void *y;  // [N][E][4]
  const int *bnd_nodes, *bnd_ghosts, *bnd_normal, *wall_idx;
  const double2 *wall_w;   // {d1, d2} per (row, slot), ghost entries zeroed
  const int2 *inv_grp;     // {first row, size} of each row's group
  const int *inv_win;      // {start, length} per (matrix, row)
  const int64_t *inv_off;  // window value offset per (matrix, row)
  const double *inv_val;
  double *gres;            // [R][E][4]
  float *ghrem;            // FP32 fields: each ghost value's remainder past its FP32 rounding,
                           // [N - Na][E][4] (or NULL)
  const uint8_t *kind;
  int64_t Na;
  int R, n, E;
  int u_shared;                // 1: u's block equals theta prime's (no wall normal to x)
  double bc_scale, theta_bar;  // dpi/dz = bc_scale * th / (theta_bar + th) on walls normal to z
};

// Sum over the wavefront (full exec mask), returned in every lane: adds of
// data-parallel moves within rows of 16 lanes (quad permutes, half-mirror,
// mirror), then the row broadcasts 15 and 31 carry the row sums to lane 63,
// which is read back. A few cycles per step, against a cross-lane permute
// through the LDS unit per step and half; one fixed order for every caller.
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROWS, 0xF, false);
  return v + __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ double wave_sum(double v) {
  v = dpp_add<0xB1, 0xF>(v);   // quad_perm 1,0,3,2
  v = dpp_add<0x4E, 0xF>(v);   // quad_perm 2,3,0,1
  v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xF>(v);  // row_mirror: every lane holds its row's sum
  v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3: lane 63 holds the total
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), 63);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), 63);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// One stencil slot's contribution to the residuals of a boundary row with
// normal `nrm`: u takes d1 on walls normal to z and d2 on walls normal to x,
// w the reverse, theta' and pi' d1. Values at ghosts count as 0 (their
// weights are zeroed as well), w at nodes on walls normal to z and u at
// nodes on walls normal to x are 0 (they are being set to 0).
template <class FT>
__device__ __forceinline__ void resid_slot(const GArgs &a, int64_t row, int k, int e, int nrm, double &ru, double &rw,
                                           double &rt, double &rp) {
  const int64_t sl = row * a.n + k;
  const int j = a.wall_idx[sl];
  const uint8_t kj = a.kind[j];
  const double2 ww = a.wall_w[sl];
  const F4<FT> f = load4(static_cast<const FT *>(a.y) + (static_cast<int64_t>(j) * a.E + e) * 4);
  const bool g = kj & KIND_GHOST;
  const double wu = nrm ? ww.y : ww.x, wv = nrm ? ww.x : ww.y;
  ru = fma(-wu, (g || (kj & KIND_XWALL)) ? 0.0 : static_cast<double>(f.v[0]), ru);
  rw = fma(-wv, (g || (kj & KIND_ZWALL)) ? 0.0 : static_cast<double>(f.v[1]), rw);
  rt = fma(-ww.x, g ? 0.0 : static_cast<double>(f.v[2]), rt);
  rp = fma(-ww.x, g ? 0.0 : static_cast<double>(f.v[3]), rp);
}

// Finish a row: boundary-condition data, the wall value set to 0, residuals out.
template <class FT>
__device__ __forceinline__ void resid_store(const GArgs &a, int64_t row, int e, int nrm, double ru, double rw,
                                            double rt, double rp) {
  FT *y = static_cast<FT *>(a.y);
  const int64_t o = (static_cast<int64_t>(a.bnd_nodes[row]) * a.E + e) * 4;
  if (nrm == 0) {
    const double thb = static_cast<double>(y[o + 2]);
    rp += a.bc_scale * thb / (a.theta_bar + thb);
    y[o + 1] = FT(0);
  } else {
    y[o + 0] = FT(0);
  }
  double *g = a.gres + (row * a.E + e) * 4;
  g[0] = ru;
  g[1] = rw;
  g[2] = rt;
  g[3] = rp;
}

// B1 part 1: boundary-row residuals r = bc - (W_I u_I + W_B u_B).
// One wavefront per (boundary row, member); lanes take stencil slots. The
// launch is short and latency-bound, so every load that does not depend on
// a gathered value is issued first: the row's normal, its wall node and that
// node's theta' (which the closure never writes), beside the slot records.
template <class FT>
__global__ __launch_bounds__(RHS_BLOCK) void ghost_resid_kernel(GArgs a) {
  const int64_t item = static_cast<int64_t>(blockIdx.x) * (RHS_BLOCK / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (item >= static_cast<int64_t>(a.R) * a.E) return;
  const int64_t row = item / a.E;
  const int e = static_cast<int>(item - row * a.E);
  FT *y = static_cast<FT *>(a.y);
  const int nrm = a.bnd_normal[row];
  const int64_t o = (static_cast<int64_t>(a.bnd_nodes[row]) * a.E + e) * 4;
  const double thb = static_cast<double>(y[o + 2]);
  double ru = 0.0, rw = 0.0, rt = 0.0, rp = 0.0;
  for (int k = lane; k < a.n; k += 64) resid_slot<FT>(a, row, k, e, nrm, ru, rw, rt, rp);
  ru = wave_sum(ru);
  rw = wave_sum(rw);
  rt = wave_sum(rt);
  rp = wave_sum(rp);
  if (lane == 0) {
    if (nrm == 0) {
      rp += a.bc_scale * thb / (a.theta_bar + thb);
      y[o + 1] = FT(0);
    } else {
      y[o + 0] = FT(0);
    }
    double *g = a.gres + (row * a.E + e) * 4;
    g[0] = ru;
    g[1] = rw;
    g[2] = rt;
    g[3] = rp;
  }
}

// One W_G^-1 row (matrix `mat`, boundary row `row`): the cyclic window of
// its group's rows that holds its kept entries.
struct InvRow {
  const double *val;
  int g0, gm, start, len;
};
__device__ __forceinline__ InvRow inv_row(const GArgs &a, int mat, int64_t row) {
  const int2 g = a.inv_grp[row];
  const int64_t slot = static_cast<int64_t>(mat) * a.R + row;
  return InvRow{a.inv_val + a.inv_off[slot], g.x, g.y, a.inv_win[2 * slot], a.inv_win[2 * slot + 1]};
}
// boundary row of window position q (< len <= gm)
__device__ __forceinline__ int64_t win_row(const InvRow &w, int q) {
  int p = w.start + q;
  if (p >= w.gm) p -= w.gm;
  return w.g0 + p;
}

// B1 part 2: ghost values u_G = W_G^-1 r through the inverse windows.
// One wavefront per (ghost row, member); lanes take window positions, two
// positions per lane at a time with both positions' loads issued before
// either is summed (the sums per lane stay in window order).
struct ApplyTerms {
  double ct, t0, t2, t3;  // theta' / pi' (and u when shared): W_G^-1 entry, residuals
  double cw, r1;          // w
  double cu, r0;          // u
};
__device__ __forceinline__ ApplyTerms apply_load(const GArgs &a, const InvRow &wt, const InvRow &ww, const InvRow &wu,
                                                 int q, int e) {
  ApplyTerms t{};
  if (q < wt.len) {
    t.ct = wt.val[q];
    const double *r = a.gres + (win_row(wt, q) * a.E + e) * 4;
    if (a.u_shared) t.t0 = r[0];
    t.t2 = r[2];
    t.t3 = r[3];
  }
  if (q < ww.len) {
    t.cw = ww.val[q];
    t.r1 = a.gres[(win_row(ww, q) * a.E + e) * 4 + 1];
  }
  if (q < wu.len) {
    t.cu = wu.val[q];
    t.r0 = a.gres[(win_row(wu, q) * a.E + e) * 4];
  }
  return t;
}
__device__ __forceinline__ void apply_sum(const GArgs &a, const InvRow &wt, const InvRow &ww, const InvRow &wu, int q,
                                          const ApplyTerms &t, double (&v)[4]) {
  if (q < wt.len) {
    if (a.u_shared) v[0] = fma(t.ct, t.t0, v[0]);
    v[2] = fma(t.ct, t.t2, v[2]);
    v[3] = fma(t.ct, t.t3, v[3]);
  }
  if (q < ww.len) v[1] = fma(t.cw, t.r1, v[1]);
  if (q < wu.len) v[0] = fma(t.cu, t.r0, v[0]);
}

template <class FT>
__global__ __launch_bounds__(RHS_BLOCK) void ghost_apply_kernel(GArgs a) {
  const int64_t item = static_cast<int64_t>(blockIdx.x) * (RHS_BLOCK / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (item >= static_cast<int64_t>(a.R) * a.E) return;
  const int64_t row = item / a.E;
  const int e = static_cast<int>(item - row * a.E);
  const int64_t go = (static_cast<int64_t>(a.bnd_ghosts[row]) * a.E + e) * 4;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const InvRow wt = inv_row(a, 2, row), ww = inv_row(a, 1, row);
  const InvRow wu = a.u_shared ? InvRow{nullptr, 0, 1, 0, 0} : inv_row(a, 0, row);
  const int L = max(max(wt.len, ww.len), wu.len);
  for (int q = lane; q < L; q += 128) {
    const ApplyTerms t0 = apply_load(a, wt, ww, wu, q, e);
    const ApplyTerms t1 = apply_load(a, wt, ww, wu, q + 64, e);
    apply_sum(a, wt, ww, wu, q, t0, v);
    apply_sum(a, wt, ww, wu, q + 64, t1, v);
  }
  for (int f = 0; f < 4; ++f) v[f] = wave_sum(v[f]);
  if (lane == 0) {
    store4(static_cast<FT *>(a.y) + go, v);
    if (a.ghrem) store_remainder(a.ghrem + go - a.Na * a.E * 4, v);
  }
}

// Ensembles (E >= GHOST_MEMBER_LANES): the same two steps with one thread
// per (boundary row, member), members in consecutive lanes, so every
// stencil slot and inverse entry is one coalesced load across the
// wavefront. Sums run in slot / entry order, so such members agree with
// single-member runs to rounding rather than bit for bit.
constexpr int GHOST_MEMBER_LANES = 16;

template <class FT>
__global__ __launch_bounds__(RHS_BLOCK) void ghost_resid_members_kernel(GArgs a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * RHS_BLOCK + threadIdx.x;
  if (t >= static_cast<int64_t>(a.R) * a.E) return;
  const int64_t row = t / a.E;
  const int e = static_cast<int>(t - row * a.E);
  const int nrm = a.bnd_normal[row];
  double ru = 0.0, rw = 0.0, rt = 0.0, rp = 0.0;
#pragma unroll 4
  for (int k = 0; k < a.n; ++k) resid_slot<FT>(a, row, k, e, nrm, ru, rw, rt, rp);
  resid_store<FT>(a, row, e, nrm, ru, rw, rt, rp);
}

template <class FT>
__global__ __launch_bounds__(RHS_BLOCK) void ghost_apply_members_kernel(GArgs a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * RHS_BLOCK + threadIdx.x;
  if (t >= static_cast<int64_t>(a.R) * a.E) return;
  const int64_t row = t / a.E;
  const int e = static_cast<int>(t - row * a.E);
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (!a.u_shared) {
    const InvRow w = inv_row(a, 0, row);
#pragma unroll 4
    for (int q = 0; q < w.len; ++q) v[0] = fma(w.val[q], a.gres[(win_row(w, q) * a.E + e) * 4], v[0]);
  }
  {
    const InvRow w = inv_row(a, 1, row);
#pragma unroll 4
    for (int q = 0; q < w.len; ++q) v[1] = fma(w.val[q], a.gres[(win_row(w, q) * a.E + e) * 4 + 1], v[1]);
  }
  {
    const InvRow w = inv_row(a, 2, row);
    if (a.u_shared) {
#pragma unroll 4
      for (int q = 0; q < w.len; ++q) {
        const double c = w.val[q];
        const double4 r = *reinterpret_cast<const double4 *>(a.gres + (win_row(w, q) * a.E + e) * 4);
        v[0] = fma(c, r.x, v[0]);
        v[2] = fma(c, r.z, v[2]);
        v[3] = fma(c, r.w, v[3]);
      }
    } else {
#pragma unroll 4
      for (int q = 0; q < w.len; ++q) {
        const double c = w.val[q];
        const double2 r = *reinterpret_cast<const double2 *>(a.gres + (win_row(w, q) * a.E + e) * 4 + 2);
        v[2] = fma(c, r.x, v[2]);
        v[3] = fma(c, r.y, v[3]);
      }
    }
  }
  const int64_t go = (static_cast<int64_t>(a.bnd_ghosts[row]) * a.E + e) * 4;
  store4(static_cast<FT *>(a.y) + go, v);
  if (a.ghrem) store_remainder(a.ghrem + go - a.Na * a.E * 4, v);
}

__global__ void misc_init_kernel(DevMisc *m, double t0) {
  m->nonfinite_step = INT_MAX;
  m->step_ctr = 0;
  m->t0 = t0;
}

__global__ void tick_kernel(DevMisc *m) { m->step_ctr += 1; }

// ---- host-side launchers ----------------------------------------------------

// Transport mirror boundary (Section 6.1): ghost k takes the value of active
// node src[k], for every member.
template <class FT>
__global__ void mirror_kernel(FT *__restrict__ y, const int *__restrict__ src, int64_t na, int64_t ng, int E) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ng * E) return;
  const int64_t k = t / E;
  const int e = static_cast<int>(t - k * E);
  y[(na + k) * E + e] = y[static_cast<int64_t>(src[k]) * E + e];
}

int launch_ghost(rbffd_ctx *ctx, rbffd_model *m, void *y) {
  if (m->physics == RBFFD_PHYS_ADVECTION && m->n_mirror > 0) {
    const int64_t cnt = m->n_mirror * m->E;
    if (m->fdt == RBFFD_F64)
      mirror_kernel<double><<<grid_for(cnt, 256), 256, 0, ctx->stream>>>(static_cast<double *>(y), m->mirror_src.as<int>(),
                                                                        m->Na, m->n_mirror, m->E);
    else
      mirror_kernel<float><<<grid_for(cnt, 256), 256, 0, ctx->stream>>>(static_cast<float *>(y), m->mirror_src.as<int>(),
                                                                       m->Na, m->n_mirror, m->E);
    RBFFD_HIP(ctx, hipGetLastError());
    return RBFFD_OK;
  }
  if (m->physics != RBFFD_PHYS_NS || m->n_bnd == 0) return RBFFD_OK;
  GArgs g{};
  g.y = y;
  g.bnd_nodes = m->bnd_nodes.as<int>();
  g.bnd_ghosts = m->bnd_ghosts.as<int>();
  g.bnd_normal = m->bnd_normal.as<int>();
  g.wall_idx = m->wall_idx.as<int>();
  g.wall_w = m->wall_w.as<double2>();
  g.inv_grp = m->inv_grp.as<int2>();
  g.inv_win = m->inv_win.as<int>();
  g.inv_off = m->inv_off.as<int64_t>();
  g.inv_val = m->inv_val.as<double>();
  g.gres = m->gres.as<double>();
  g.ghrem = m->ghrem.as<float>();
  g.Na = m->Na;
  g.kind = m->kind.as<uint8_t>();
  g.R = m->n_bnd;
  g.u_shared = m->u_shares_tp;
  g.n = m->n;
  g.E = m->E;
  g.bc_scale = m->g / (m->c_p * m->theta_bar);
  g.theta_bar = m->theta_bar;
  const int64_t cnt = static_cast<int64_t>(m->n_bnd) * m->E;
  if (m->E >= GHOST_MEMBER_LANES) {                                       // one thread each
    const unsigned grid = grid_for(cnt, RHS_BLOCK);
    if (m->fdt == RBFFD_F64) {
      ghost_resid_members_kernel<double><<<grid, RHS_BLOCK, 0, ctx->stream>>>(g);
      ghost_apply_members_kernel<double><<<grid, RHS_BLOCK, 0, ctx->stream>>>(g);
    } else {
      ghost_resid_members_kernel<float><<<grid, RHS_BLOCK, 0, ctx->stream>>>(g);
      ghost_apply_members_kernel<float><<<grid, RHS_BLOCK, 0, ctx->stream>>>(g);
    }
  } else {
    const unsigned grid = grid_for(cnt, RHS_BLOCK / 64);                 // one wavefront each
    if (m->fdt == RBFFD_F64) {
      ghost_resid_kernel<double><<<grid, RHS_BLOCK, 0, ctx->stream>>>(g);
      ghost_apply_kernel<double><<<grid, RHS_BLOCK, 0, ctx->stream>>>(g);
    } else {
      ghost_resid_kernel<float><<<grid, RHS_BLOCK, 0, ctx->stream>>>(g);
      ghost_apply_kernel<float><<<grid, RHS_BLOCK, 0, ctx->stream>>>(g);
    }
  }
  RBFFD_HIP(ctx, hipGetLastError());
  return RBFFD_OK;
}

// One stage-kernel launch. With events (kernel timing), the launch goes
// through hipExtLaunchKernel, which stamps them with the kernel's own start
// and end, so the measured time leaves out the dispatch around it.
template <class A>
hipError_t launch_timed(void (*k)(A), unsigned grid, unsigned block, hipStream_t st, const A &a, hipEvent_t e0,
                        hipEvent_t e1) {
  if (e0) {
    A copy = a;
    void *args[] = {&copy};
    return hipExtLaunchKernel(reinterpret_cast<const void *>(k), dim3(grid), dim3(block), args, 0, st, e0, e1, 0);
  }
  k<<<grid, block, 0, st>>>(a);
  return hipGetLastError();
}

template <class FT, int WDT, int S>
hipError_t launch_ns_one(int64_t cnt, hipStream_t st, const NSArgs &a, hipEvent_t e0, hipEvent_t e1) {
  constexpr int B = StageShape<S>::block;
  if (a.E % 64 == 0) return launch_timed(ns_stage_kernel<FT, WDT, S, true>, grid_for(cnt, B), B, st, a, e0, e1);
  return launch_timed(ns_stage_kernel<FT, WDT, S, false>, grid_for(cnt, B), B, st, a, e0, e1);
}

template <class FT, int WDT>
hipError_t launch_ns_shape(int shape, int64_t cnt, hipStream_t st, const NSArgs &a, hipEvent_t e0, hipEvent_t e1) {
  switch (shape) {
    case 0: return launch_ns_one<FT, WDT, 0>(cnt, st, a, e0, e1);
    case 1: return launch_ns_one<FT, WDT, 1>(cnt, st, a, e0, e1);
    case 2: return launch_ns_one<FT, WDT, 2>(cnt, st, a, e0, e1);
    case 3: return launch_ns_one<FT, WDT, 3>(cnt, st, a, e0, e1);
    case 4: return launch_ns_one<FT, WDT, 4>(cnt, st, a, e0, e1);
    default: return launch_ns_one<FT, WDT, 5>(cnt, st, a, e0, e1);
  }
}

struct StageSpec {
  const void *ys, *yn;
  void *out;
  double ca, cb, t_off;
  int mode, acc_mode, check;
};

int launch_stage(rbffd_ctx *ctx, rbffd_model *m, const StageSpec &sp, double t_fixed, bool use_misc, double dt) {
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (m->profile) {
    RBFFD_HIP(ctx, hipEventCreate(&ev0));
    if (hipEventCreate(&ev1) != hipSuccess) {
      (void)hipEventDestroy(ev0);
      return rbffd_fail(ctx, RBFFD_EDEVICE, "hipEventCreate failed");
    }
    m->prof_events.push_back({ev0, ev1});
  }
  const int64_t cnt = m->Na * m->E;
  DevMisc *misc = m->dev_misc.as<DevMisc>();
  if (m->physics == RBFFD_PHYS_NS) {
    NSArgs a{};
    a.ys = sp.ys;
    a.yn = sp.yn;
    a.out = sp.out;
    a.acc = m->acc.p;
    a.idx_t = m->idx_t.as<int>() + m->k0 * m->Na;  // stream slot k is stencil slot k0 + k
    a.off16 = m->off16.as<int16_t>();
    a.aux32 = m->aux32.as<uint32_t>();
    a.rec = m->rec.p;
    a.rec2 = m->rec2.p;
    a.kind = m->kind.as<uint8_t>();
    a.pibar = m->pibar.as<double>();
    a.order = m->use_order ? m->order.as<int>() : nullptr;
    a.rec_t = m->use_order ? m->rec_order.p : nullptr;
    a.ghrem = m->ghrem.as<float>();
    a.Na = m->Na;
    a.n = m->n - m->k0;
    a.E = m->E;
    a.c_p = m->c_p;
    a.rcv = m->R_d / m->c_v;
    a.g = m->g;
    a.theta_bar = m->theta_bar;
    a.mu = m->mu;
    a.hv = m->hv_coeff;
    a.dpibar = -m->g / (m->c_p * m->theta_bar);
    a.u_bar = m->u_bar;
    a.ca = sp.ca;
    a.cb = sp.cb;
    a.mode = sp.mode;
    a.acc_mode = sp.acc_mode;
    a.misc = misc;
    a.check = sp.check;
    const int shape = m->shape >= 0 ? m->shape : default_shape(m->wdt);
    if (m->fdt == RBFFD_F64)
      RBFFD_HIP(ctx, (launch_ns_shape<double, RBFFD_F64>(shape, cnt, ctx->stream, a, ev0, ev1)));
    else if (m->wdt == RBFFD_F32)
      RBFFD_HIP(ctx, (launch_ns_shape<float, RBFFD_F32>(shape, cnt, ctx->stream, a, ev0, ev1)));
    else
      RBFFD_HIP(ctx, (launch_ns_shape<float, RBFFD_BF16>(shape, cnt, ctx->stream, a, ev0, ev1)));
  } else {
    AdvArgs a{};
    a.ys = sp.ys;
    a.yn = sp.yn;
    a.out = sp.out;
    a.acc = m->acc.p;
    a.idx_t = m->idx_t.as<int>();
    a.rec = m->rec.as<RecAdv>();
    a.Na = m->Na;
    a.n = m->n;
    a.E = m->E;
    a.hv = m->hv_coeff;
    a.omega = M_PI / m->vel_period;
    a.t_fixed = t_fixed;
    a.t_off = sp.t_off;
    a.dt = dt;
    a.ca = sp.ca;
    a.cb = sp.cb;
    a.mode = sp.mode;
    a.acc_mode = sp.acc_mode;
    a.misc = use_misc ? misc : nullptr;
    a.check = sp.check;
    if (sp.mode != 0 && m->n_mirror > 0) {
      a.mir_off = m->mirror_off.as<int>();
      a.mir_list = m->mirror_list.as<int>();
    }
    if (m->fdt == RBFFD_F64)
      RBFFD_HIP(ctx, launch_timed(adv_stage_kernel<double>, grid_for(cnt, RHS_BLOCK), RHS_BLOCK, ctx->stream, a, ev0, ev1));
    else
      RBFFD_HIP(ctx, launch_timed(adv_stage_kernel<float>, grid_for(cnt, RHS_BLOCK), RHS_BLOCK, ctx->stream, a, ev0, ev1));
  }
  return RBFFD_OK;
}

// Zero the ghost rows of a tendency / state buffer (fill kernel, graph-safe).
__global__ void zero_rows_kernel(void *p, int64_t first_byte, int64_t n_bytes) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n_bytes / 4) static_cast<uint32_t *>(p)[first_byte / 4 + t] = 0u;
}

// Whether a stage's input needs the boundary launch first: always for the
// Navier-Stokes closure; for transport only the step's input, since every
// stage update writes its mirror ghosts itself.
bool needs_ghost(const rbffd_model *m, const StageSpec &sp, const void *y) {
  return m->physics != RBFFD_PHYS_ADVECTION || sp.ys == y;
}

// One full time step, as a sequence of launches on the context stream.
int enqueue_step(rbffd_ctx *ctx, rbffd_model *m, void *y, double dt, int tableau) {
  int rc;
  void *ya = m->ya.p, *yb = m->yb.p;
  if (tableau == RBFFD_RK4) {
    const StageSpec st[4] = {
        {y, y, ya, 0.5 * dt, dt / 6.0, 0.0, 1, 1, 0},
        {ya, y, yb, 0.5 * dt, dt / 3.0, 0.5 * dt, 1, 2, 0},
        {yb, y, ya, dt, dt / 3.0, 0.5 * dt, 1, 2, 0},
        {ya, nullptr, y, dt / 6.0, 0.0, dt, 2, 0, 1},
    };
    for (const StageSpec &sp : st) {
      if (needs_ghost(m, sp, y) && (rc = launch_ghost(ctx, m, const_cast<void *>(sp.ys)))) return rc;
      if ((rc = launch_stage(ctx, m, sp, 0.0, true, dt))) return rc;
    }
  } else {
    const StageSpec st[3] = {
        {y, y, ya, dt / 3.0, 0.0, 0.0, 1, 0, 0},
        {ya, y, yb, dt / 2.0, 0.0, dt / 3.0, 1, 0, 0},
        {yb, y, y, dt, 0.0, dt / 2.0, 1, 0, 1},
    };
    for (const StageSpec &sp : st) {
      if (needs_ghost(m, sp, y) && (rc = launch_ghost(ctx, m, const_cast<void *>(sp.ys)))) return rc;
      if ((rc = launch_stage(ctx, m, sp, 0.0, true, dt))) return rc;
    }
  }
  tick_kernel<<<1, 1, 0, ctx->stream>>>(m->dev_misc.as<DevMisc>());
  RBFFD_HIP(ctx, hipGetLastError());
  return RBFFD_OK;
}

}  // namespace

int model_ghost(rbffd_ctx *ctx, rbffd_model *m, void *state) { return launch_ghost(ctx, m, state); }

int model_rhs(rbffd_ctx *ctx, rbffd_model *m, double t, void *state, void *tendency) {
  int rc = launch_ghost(ctx, m, state);
  if (rc) return rc;
  StageSpec sp{state, state, tendency, 0.0, 0.0, 0.0, 0, 0, 0};
  rc = launch_stage(ctx, m, sp, t, false, 0.0);
  if (rc) return rc;
  if (m->N > m->Na) {
    const int64_t row = static_cast<int64_t>(m->E) * m->F * m->field_bytes();
    const int64_t first = m->Na * row, bytes = (m->N - m->Na) * row;
    zero_rows_kernel<<<grid_for(bytes / 4, 256), 256, 0, ctx->stream>>>(tendency, first, bytes);
    RBFFD_HIP(ctx, hipGetLastError());
  }
  return RBFFD_OK;
}

namespace {

// Steps per replay of the larger captured graph: consecutive graph launches
// leave the device idle for about 8 us, so a run replays GRAPH_STEPS steps per
// launch and single steps for the remainder.
constexpr int GRAPH_STEPS = 8;

void drop_graphs(rbffd_model *m) {
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  if (m->exec_n) (void)hipGraphExecDestroy(m->exec_n);
  if (m->graph_n) (void)hipGraphDestroy(m->graph_n);
  m->exec = m->exec_n = nullptr;
  m->graph = m->graph_n = nullptr;
}

// Captures k steps into one graph and instantiates it.
int capture_steps(rbffd_ctx *ctx, rbffd_model *m, void *state, double dt, int tableau, int k, hipGraph_t *graph_out,
                  hipGraphExec_t *exec_out) {
  hipStream_t cs = ctx->stream;
  bool own_stream = false;
  if (cs == nullptr) {  // the null stream cannot be captured
    RBFFD_HIP(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    own_stream = true;
  }
  hipStream_t saved = ctx->stream;
  ctx->stream = cs;
  hipError_t eb = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  int rc = RBFFD_OK;
  hipGraph_t graph = nullptr;
  hipError_t ec = eb;
  if (eb == hipSuccess) {
    for (int i = 0; i < k && rc == RBFFD_OK; ++i) rc = enqueue_step(ctx, m, state, dt, tableau);
    ec = hipStreamEndCapture(cs, &graph);
  }
  ctx->stream = saved;
  if (own_stream) (void)hipStreamDestroy(cs);
  if (rc || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc ? rc : rbffd_fail(ctx, RBFFD_EDEVICE, "graph capture: %s", hipGetErrorString(ec));
  }
  *graph_out = graph;
  RBFFD_HIP(ctx, hipGraphInstantiate(exec_out, graph, nullptr, nullptr, 0));
  return RBFFD_OK;
}

}  // namespace

int model_step(rbffd_ctx *ctx, rbffd_model *m, void *state, double *t, double dt, int64_t n_steps, int tableau) {
  if (n_steps == 0) return RBFFD_OK;
  hipStream_t s = ctx->stream;
  misc_init_kernel<<<1, 1, 0, s>>>(m->dev_misc.as<DevMisc>(), *t);
  RBFFD_HIP(ctx, hipGetLastError());
  if (m->profile) {
    for (int64_t k = 0; k < n_steps; ++k) {
      int rc = enqueue_step(ctx, m, state, dt, tableau);
      if (rc) return rc;
    }
  } else {
    // graphs are captured for one (state, dt, tableau) and only when a call
    // needs them: the eight-step graph for n_steps >= 8, the one-step graph
    // for a remainder
    if (m->graph_state != state || m->graph_dt != dt || m->graph_tableau != tableau) {
      drop_graphs(m);
      m->graph_state = state;
      m->graph_dt = dt;
      m->graph_tableau = tableau;
    }
    int rc = RBFFD_OK;
    if (n_steps >= GRAPH_STEPS && !m->exec_n)
      rc = capture_steps(ctx, m, state, dt, tableau, GRAPH_STEPS, &m->graph_n, &m->exec_n);
    if (rc == RBFFD_OK && n_steps % GRAPH_STEPS != 0 && !m->exec)
      rc = capture_steps(ctx, m, state, dt, tableau, 1, &m->graph, &m->exec);
    if (rc) {
      drop_graphs(m);
      m->graph_state = nullptr;
      return rc;
    }
    int64_t k = 0;
    for (; k + GRAPH_STEPS <= n_steps; k += GRAPH_STEPS) RBFFD_HIP(ctx, hipGraphLaunch(m->exec_n, s));
    for (; k < n_steps; ++k) RBFFD_HIP(ctx, hipGraphLaunch(m->exec, s));
  }
  DevMisc h{};
  RBFFD_HIP(ctx, hipMemcpyAsync(&h, m->dev_misc.p, sizeof(h), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  const double t0 = *t;
  *t = t0 + static_cast<double>(n_steps) * dt;
  if (h.nonfinite_step != INT_MAX)
    return rbffd_fail(ctx, RBFFD_ENONFINITE, "non-finite state at step %d of this call", h.nonfinite_step + 1);
  return RBFFD_OK;
}

int model_profile(rbffd_model *m, int enable) {
  m->profile = enable ? 1 : 0;
  return RBFFD_OK;
}

int model_profile_read(rbffd_model *m, double *total_ms, int64_t *launches) {
  rbffd_ctx *ctx = m->ctx;
  RBFFD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double sum = 0.0;
  for (auto &p : m->prof_events) {
    float ms = 0.0f;
    RBFFD_HIP(ctx, hipEventElapsedTime(&ms, p.first, p.second));
    sum += ms;
  }
  *total_ms = sum;
  *launches = static_cast<int64_t>(m->prof_events.size());
  for (auto &p : m->prof_events) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  m->prof_events.clear();
  return RBFFD_OK;
}

namespace {
__global__ __launch_bounds__(256) void stream_copy_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                          int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}
}  // namespace

int stream_copy(rbffd_ctx *ctx, void *dst, const void *src, int64_t bytes) {
  const int64_t n = bytes / 16;
  if (n == 0) return RBFFD_OK;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(grid_for(n, 256), 65536));
  stream_copy_kernel<<<grid, 256, 0, ctx->stream>>>(static_cast<uint4 *>(dst), static_cast<const uint4 *>(src), n);
  RBFFD_HIP(ctx, hipGetLastError());
  return RBFFD_OK;
}

// Time every launch shape of the stage kernel on this model's data (a few
// tendency evaluations of `state` into the model's stage buffer, HIP events
// on the context stream) and keep the fastest.
int model_tune(rbffd_ctx *ctx, rbffd_model *m, void *state, int *chosen, double *best_us) {
  if (m->physics != RBFFD_PHYS_NS) {
    *chosen = -1;
    *best_us = 0.0;
    return RBFFD_OK;
  }
  // member-wavefront models also try the Morton traversal
  const int n_orders = m->order.p ? 2 : 1;
  const int forced = *chosen;
  if (forced < -1 || forced >= kNumShapes * n_orders)
    return rbffd_fail(ctx, RBFFD_EINVAL, "model_tune: shape %d is not -1 or in [0, %d)", forced,
                      kNumShapes * n_orders);
  const int saved_profile = m->profile;
  m->profile = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = RBFFD_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = rbffd_fail(ctx, RBFFD_EDEVICE, "model_tune: hipEventCreate failed");
  if (rc == RBFFD_OK) rc = launch_ghost(ctx, m, state);
  double best = 1e300;
  int best_s = default_shape(m->wdt), best_o = 0;
  StageSpec sp{state, state, m->ya.p, 0.0, 0.0, 0.0, 0, 0, 0};
  for (int o = 0; o < n_orders && rc == RBFFD_OK; ++o) {
    m->use_order = o;
    for (int sh = 0; sh < kNumShapes && rc == RBFFD_OK; ++sh) {
      if (forced >= 0 && forced != sh + kNumShapes * o) continue;
      m->shape = sh;
      rc = launch_stage(ctx, m, sp, 0.0, false, 0.0);  // warm-up
      if (rc) break;
      float ms = 0.0f;
      constexpr int reps = 5;
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) rc = rbffd_fail(ctx, RBFFD_EDEVICE, "hipEventRecord failed");
      for (int r = 0; r < reps && rc == RBFFD_OK; ++r) rc = launch_stage(ctx, m, sp, 0.0, false, 0.0);
      if (rc == RBFFD_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = rbffd_fail(ctx, RBFFD_EDEVICE, "model_tune: event timing failed");
      if (rc) break;
      const double us = 1e3 * ms / reps;
      if (us < best) {
        best = us;
        best_s = sh;
        best_o = o;
      }
    }
  }
  m->use_order = best_o;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  m->shape = best_s;
  m->profile = saved_profile;
  drop_graphs(m);  // a captured graph holds the old shape
  *chosen = best_s + kNumShapes * best_o;
  *best_us = best;
  return rc;
}

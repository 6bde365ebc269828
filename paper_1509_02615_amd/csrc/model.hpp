// The right-hand-side model: device-resident, slot-major copies of the
// differentiation matrices plus the ghost-closure operators and RK buffers.
#pragma once

#include "common.hpp"

// Weight records, slot-major: record (k, i) holds slot k of node i. The
// neighbour index j of a Navier-Stokes record travels as the 16-bit offset
// j - i (int16 [n][Na], inline in the BF16 record); an offset outside
// +-32767 (a ghost neighbour: ghosts are stored after the active nodes) is
// OFF_FAR, and the kernel then reads j from the full index array idx_t.
constexpr int16_t OFF_FAR = -32768;
struct RecF64 {      // FP64 Navier-Stokes: Dx, Dz, Lap, Lap^k
  double dx, dz, lap, hv;
};
struct RecF32 {      // FP32 Navier-Stokes: Dx, Dz, Lap and Lap^k, each the FP32 rounding hi
  float dx, dz, lap, hv;  // of the FP64 weight
};
// The FP32 layout's second stream, one 32-bit word per record: bits 31-16
// the neighbour offset; bits 15-10, 9-5 and 4-0 signed corrections q of the
// Lap^k, Dx and Dz weights, each weight being hi (1 + q s) with s = 2^-29
// (Lap^k, within about 2^-30 of the FP64 weight) and 2^-28 (Dx, Dz, within
// about 2^-29). The corrected Dx and Dz weights enter only the divergence
// u_x + w_z, which the stage kernel sums in FP64: the pressure tendency is
// the small difference of that term and w dpi-bar/dz in a developed flow.
constexpr double HV_Q_SCALE = 0x1p-29;
constexpr double D_Q_SCALE = 0x1p-28;
constexpr int HV_Q_BITS = 6, D_Q_BITS = 5;
struct RecMW {       // ensembles of 64k members (one record per wavefront of 64 members,
  double dx, dz, hv; // through the scalar cache: bytes per member are negligible, so the
  float lap;         // weights the FP64 sums take stay FP64 and the full index is inline;
  int idx;           // one aligned 32-byte scalar load per slot)
};
struct RecBF16 {     // BF16 Navier-Stokes: Dx, Dz, Lap (bfloat16 bits) and the offset
  uint16_t dx, dz, lap;
  int16_t off;
};
struct RecBF16X {    // the BF16 layout's second stream: the Lap^k weight as FP32 hi with
  float hv;          // an 8-bit correction (hv (1 + hvq 2^-31), about 2^-32), and 8-bit
  int8_t hvq, lapq;  // corrections of the Lap, Dx and Dz weights, each bf16 (1 + q 2^-15),
  int8_t dxq, dzq;   // so that they keep about 16 significant bits
};
constexpr double HV_Q8_SCALE = 0x1p-31;
constexpr float BF_Q_SCALE = 0x1p-15f;
struct RecAdv {      // transport: folded flux weights and Lap^k
  double adv, hv;
};

// Node kinds (bits): on a wall normal to z (w = 0), ghost, on a wall normal
// to x (u = 0); a corner of a closed box carries both wall bits. An active
// node whose stencil holds a ghost also carries KIND_REACH.
constexpr uint8_t KIND_ZWALL = 1, KIND_GHOST = 2, KIND_XWALL = 4, KIND_REACH = 8;

struct rbffd_model {
  rbffd_ctx *ctx = nullptr;
  int physics = 0, fdt = RBFFD_F64, wdt = RBFFD_F64;
  int n = 0, E = 1, F = 1;
  int64_t N = 0, Na = 0;
  // slot-major differentiation matrices
  DevBuf idx_t;     // int32 [n][Na] full neighbour indices
  DevBuf off16;     // int16 [n - k0][Na] neighbour offsets j - i (F64 layout)
  DevBuf aux32;     // uint32 [n - k0][Na] neighbour offset and weight corrections (FP32 layout)
  bool wide_rec = false;  // FP32 records carry the full index (RecMW)
  int k0 = 0;             // first slot in the stream (1: every stencil starts with its centre, which
                          // centre-subtracted sums skip); the stream arrays hold slots k0..n-1
  DevBuf rec;       // RecF64 / RecF32 / RecMW / RecBF16 [n - k0][Na], RecAdv [n][Na]
  DevBuf rec2;      // RecBF16X [n - k0][Na] (BF16 layout)
  DevBuf rec_order; // RecMW [n - k0][Na] in the Morton traversal's order (FP32 ensembles)
  DevBuf kind;      // uint8 [N]: KIND_* bits (0: interior)
  DevBuf order;     // int32 [Na]: Morton traversal order of the member-wavefront stage kernel
  int use_order = 0;  // traverse in `order` (chosen by the tuner) instead of node order
  DevBuf pibar;     // double [Na]
  double hv_coeff = 0.0, vel_period = 1.0;
  double c_p = 0, c_v = 0, R_d = 0, g = 0, theta_bar = 0, mu = 0, u_bar = 0;
  // ghost closure over R boundary rows
  int n_bnd = 0, inv_max_row = 0;
  int u_shares_tp = 0;             // no wall normal to x: u's W_G equals theta prime's
  // (rows reordered so that each group of rows sharing ghosts is contiguous)
  DevBuf bnd_nodes, bnd_ghosts;    // int32 [R]
  DevBuf bnd_normal;               // int32 [R]: 0 wall normal to z, 1 normal to x
  DevBuf wall_idx;                 // int32 [R][n] the rows' stencils
  DevBuf wall_w;                   // double2 {d1, d2} [R][n], ghost entries zeroed
  DevBuf inv_grp;                  // int2 [R] {first row, size} of the row's group
  DevBuf inv_win;                  // int [3][R][2] {start, length} of each W_G^-1 row's cyclic
                                   // window within the group (u, w, theta'/pi')
  DevBuf inv_off;                  // int64 [3][R] offset of the window's values
  DevBuf inv_val;                  // double: window values
  DevBuf gres;                     // double [R][E][4] residuals
  DevBuf ghrem;                    // float [N - Na][E][4]: the last closure's ghost values' FP64
                                   // remainders past their FP32 rounding in the state (FP32 fields)
  // transport mirror ghosts
  int64_t n_mirror = 0;
  DevBuf mirror_src;               // int32 [N - Na]
  DevBuf mirror_off, mirror_list;  // per active node, its ghosts k (node Na + k): list[off[i] .. off[i+1])
  // time stepping
  DevBuf ya, yb, acc;              // [N][E][F] stage buffers
  DevBuf dev_misc;                 // {int nonfinite_step, int step_ctr, double t0}
  hipGraph_t graph = nullptr;      // one captured step
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph_n = nullptr;    // GRAPH_STEPS captured steps
  hipGraphExec_t exec_n = nullptr;
  void *graph_state = nullptr;
  double graph_dt = 0.0;
  int graph_tableau = -1;
  int64_t bytes_per_node = 0;
  int shape = -1;  // stage-kernel launch shape (-1: the precision's default)
  // kernel timing (measurement only)
  int profile = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;

  size_t field_bytes() const { return fdt == RBFFD_F64 ? 8 : 4; }
  size_t state_bytes() const { return static_cast<size_t>(N) * E * F * field_bytes(); }
};

struct DevMisc {
  int nonfinite_step;
  int step_ctr;
  double t0;
};

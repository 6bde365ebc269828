// The right-hand-side model: device-resident, slot-major copies of the
// differentiation matrices plus the ghost-closure operators and RK buffers.
#pragma once

#include "common.hpp"

// Weight records, slot-major: record (k, i) holds slot k of node i.
struct RecF64 {      // FP64 Navier-Stokes: Dx, Dz, Lap, Lap^k
  double dx, dz, lap, hv;
};
struct RecF32 {      // FP32 Navier-Stokes: Dx, Dz, Lap and the neighbour index
  float dx, dz, lap;
  int idx;
};
struct RecBF16 {     // BF16 Navier-Stokes: Dx, Dz, Lap (bfloat16 bits) and the index
  uint16_t dx, dz, lap, pad;
  int idx;
};
struct RecAdv {      // transport: folded flux weights and Lap^k
  double adv, hv;
};

struct rbffd_model {
  rbffd_ctx *ctx = nullptr;
  int physics = 0, fdt = RBFFD_F64, wdt = RBFFD_F64;
  int n = 0, E = 1, F = 1;
  int64_t N = 0, Na = 0;
  // slot-major differentiation matrices
  DevBuf idx_t;     // int32 [n][Na] (F64 and transport layouts)
  DevBuf rec;       // RecF64 / RecF32 / RecBF16 / RecAdv [n][Na]
  DevBuf hv_t;      // double [n][Na] (F32 / BF16 layouts)
  DevBuf kind;      // uint8 [N]: 0 interior, 1 wall, 2 ghost
  DevBuf pibar;     // double [Na]
  double hv_coeff = 0.0, vel_period = 1.0;
  double c_p = 0, c_v = 0, R_d = 0, g = 0, theta_bar = 0, mu = 0, u_bar = 0;
  // ghost closure
  int n_walls = 0, nb = 0, band = 0;
  DevBuf wall_nodes, ghost_nodes;  // int32 [n_walls][nb]
  DevBuf wall_idx;                 // int32 [n_walls][nb][n]
  DevBuf wall_w;                   // double2 {dz, dzz} [n_walls][nb][n], ghost entries zeroed
  DevBuf ginv;                     // double [n_walls][2][nb][band]  (0: Dz, 1: Dzz)
  DevBuf gstart;                   // int32 [n_walls][2][nb]
  DevBuf gres;                     // double [n_walls][nb][E][4]
  // time stepping
  DevBuf ya, yb, acc;              // [N][E][F] stage buffers
  DevBuf dev_misc;                 // {int nonfinite_step, int step_ctr, double t0}
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
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

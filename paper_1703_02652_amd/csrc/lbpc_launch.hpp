// Host-side launchers of the per-format kernels.  Each kernel translation unit
// includes this file once and instantiates the launchers for one format.
#pragma once
#include "lbpc_adjoint.hpp"
#include "lbpc_device.hpp"

namespace lbpc {

inline dim3 cell_grid(int64_t n) { return dim3(static_cast<unsigned>((n + 255) / 256)); }

// Workgroups for ntiles tiles: one per tile, or a persistent grid rounded up to
// a multiple of kXcds (workgroup b then keeps to queue positions equal to b
// modulo kXcds, which the dispatcher sends to one XCD).
inline int step_grid(int ntiles, int grid) {
  if (grid <= 0) return ntiles;
  const int g = grid < ntiles ? grid : ntiles;
  return (g + kXcds - 1) / kXcds * kXcds;
}

template <int P>
hipError_t launch_step(const StepArgs& a) {
  if (a.ntiles <= 0) return hipSuccess;
  const dim3 grid(step_grid(a.ntiles, a.grid));
  const dim3 block(a.block);
#define LBPC_STEP(FL, MR, BU)                                                              \
  hipLaunchKernelGGL((k_step<P, FL, MR, BU>), grid, block, 0, a.stream, a.cavs, a.tiles,  \
                     a.ntiles, a.reverse, a.src, a.dst, a.partials, a.sums, a.status)
#define LBPC_STEP_B(FL, MR)                                    \
  do {                                                         \
    if (a.budget == 2) LBPC_STEP(FL, MR, 2);                   \
    else if (a.budget == 1) LBPC_STEP(FL, MR, 1);              \
    else LBPC_STEP(FL, MR, 0);                                 \
  } while (0)
  if (a.flow) {
    if (a.mrt) LBPC_STEP_B(true, true); else LBPC_STEP_B(true, false);
  } else {
    if (a.mrt) LBPC_STEP_B(false, true); else LBPC_STEP_B(false, false);
  }
#undef LBPC_STEP_B
#undef LBPC_STEP
  return hipGetLastError();
}

template <int P>
hipError_t launch_init(const CavParams* cavs, const int2* tiles, int ntiles, int block, int flow,
                       char* dst, const double* T0, hipStream_t st) {
  if (flow)
    hipLaunchKernelGGL((k_init<P, true>), dim3(ntiles), dim3(block), 0, st, cavs, tiles, ntiles, dst, T0);
  else
    hipLaunchKernelGGL((k_init<P, false>), dim3(ntiles), dim3(block), 0, st, cavs, tiles, ntiles, dst, T0);
  return hipGetLastError();
}

template <int P>
hipError_t launch_measure(const CavParams* cavs, const int2* tiles, int ntiles, int block,
                          int flow, int mrt, const char* src, double* partials, hipStream_t st) {
#define LBPC_MEAS(FL, MR)                                                                     \
  hipLaunchKernelGGL((k_measure<P, FL, MR>), dim3(ntiles), dim3(block), 0, st, cavs, tiles,   \
                     ntiles, src, partials)
  if (flow) { if (mrt) LBPC_MEAS(true, true); else LBPC_MEAS(true, false); }
  else { if (mrt) LBPC_MEAS(false, true); else LBPC_MEAS(false, false); }
#undef LBPC_MEAS
  return hipGetLastError();
}

template <int P>
hipError_t launch_fields(const CavParams* cav, int64_t n, int flow, const char* src,
                         uint32_t mask, double* out, hipStream_t st) {
  if (flow) hipLaunchKernelGGL((k_fields<P, true>), cell_grid(n), dim3(256), 0, st, cav, src, mask, out);
  else hipLaunchKernelGGL((k_fields<P, false>), cell_grid(n), dim3(256), 0, st, cav, src, mask, out);
  return hipGetLastError();
}

template <int P>
hipError_t launch_get_state(const CavParams* cav, int64_t n, int flow, const char* src,
                            double* f, double* g, hipStream_t st) {
  if (flow) hipLaunchKernelGGL((k_get_state<P, true>), cell_grid(n), dim3(256), 0, st, cav, src, f, g);
  else hipLaunchKernelGGL((k_get_state<P, false>), cell_grid(n), dim3(256), 0, st, cav, src, f, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_set_state(const CavParams* cav, int64_t n, int flow, char* dst,
                            const double* f, const double* g, hipStream_t st) {
  if (flow) hipLaunchKernelGGL((k_set_state<P, true>), cell_grid(n), dim3(256), 0, st, cav, dst, f, g);
  else hipLaunchKernelGGL((k_set_state<P, false>), cell_grid(n), dim3(256), 0, st, cav, dst, f, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_adjoint(const AdjArgs& a) {
  const dim3 grid(step_grid(a.ntiles, 0)), block(a.block);
#define LBPC_ADJ(FL, MR)                                                                    \
  hipLaunchKernelGGL((k_adjoint<P, FL, MR>), grid, block, 0, a.stream, a.cavs, a.tiles,    \
                     a.ntiles, a.reverse, a.last, a.state, a.lam_in, a.lam_out, a.dTw)
  if (a.flow) { if (a.mrt) LBPC_ADJ(true, true); else LBPC_ADJ(true, false); }
  else { if (a.mrt) LBPC_ADJ(false, true); else LBPC_ADJ(false, false); }
#undef LBPC_ADJ
  return hipGetLastError();
}

template <int P>
hipError_t launch_adj_seed(const CavParams* cav, int64_t n, int flow, double scale,
                           const char* state, char* lam, double* dTw, hipStream_t st) {
  if (flow) hipLaunchKernelGGL((k_adj_seed<P, true>), cell_grid(n), dim3(256), 0, st, cav, state, lam, scale, dTw);
  else hipLaunchKernelGGL((k_adj_seed<P, false>), cell_grid(n), dim3(256), 0, st, cav, state, lam, scale, dTw);
  return hipGetLastError();
}

template <int P>
hipError_t launch_adj_T0(const CavParams* cav, int64_t n, int flow, const char* state0,
                         const char* lam, double* out, hipStream_t st) {
  if (flow) hipLaunchKernelGGL((k_adj_T0<P, true>), cell_grid(n), dim3(256), 0, st, cav, state0, lam, out);
  else hipLaunchKernelGGL((k_adj_T0<P, false>), cell_grid(n), dim3(256), 0, st, cav, state0, lam, out);
  return hipGetLastError();
}

#define LBPC_INSTANTIATE(P)                                                                       \
  template hipError_t launch_step<P>(const StepArgs&);                                            \
  template hipError_t launch_init<P>(const CavParams*, const int2*, int, int, int, char*,         \
                                     const double*, hipStream_t);                                 \
  template hipError_t launch_measure<P>(const CavParams*, const int2*, int, int, int, int,        \
                                        const char*, double*, hipStream_t);                       \
  template hipError_t launch_fields<P>(const CavParams*, int64_t, int, const char*, uint32_t,     \
                                       double*, hipStream_t);                                     \
  template hipError_t launch_get_state<P>(const CavParams*, int64_t, int, const char*, double*,   \
                                          double*, hipStream_t);                                  \
  template hipError_t launch_set_state<P>(const CavParams*, int64_t, int, char*, const double*,   \
                                          const double*, hipStream_t);                            \
  template hipError_t launch_adjoint<P>(const AdjArgs&);                                          \
  template hipError_t launch_adj_seed<P>(const CavParams*, int64_t, int, double, const char*,     \
                                         char*, double*, hipStream_t);                            \
  template hipError_t launch_adj_T0<P>(const CavParams*, int64_t, int, const char*, const char*,  \
                                       double*, hipStream_t);

}  // namespace lbpc

// Internal interface between the runtime (lbpc_runtime.hip) and the kernel
// translation units (one per storage format).  Plain data only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbpc {

enum Prec { P64 = 0, P32 = 1, P16 = 2, PB16 = 3 };
enum Bc { BC_PERIODIC = 0, BC_DIRICHLET = 1, BC_ADIABATIC = 2 };

// Per-cavity constants in the compute type of a kernel (precomputed on the
// host so that kernels do not convert them per workgroup).
template <class R> struct Pars {
  R fshift, g_beta_rho0, T_ref;
  R s_nu, s_e, s_eps, s_q, s_pi, s_t;
  R lam_s, dlam, inv_rcw;       // lambda(f_l) = lam_s + f_l dlam
  R cp_s, dcp;                  // C_p(f_l) = cp_s + f_l dcp
  R w3, w21, whalf, wabb;       // 3, 21, 1/2 and 1 times omega_T C_p,ref
  R gshift;                     // (omega_T / 2) C_p,ref T_shift (16-bit formats), else 0
  R sig_ovr[7];
};

// Per-cavity constants, read by every workgroup of that cavity through scalar
// loads (the cavity index of a tile is uniform across the workgroup).
struct alignas(16) CavParams {
  int32_t nx, ny, nz, n;        // n = nx * ny * nz (< 2^31)
  int32_t nxy;
  int32_t bc[6];
  int32_t tile0, ntiles;        // this cavity's tiles in the tile queue
  int32_t chunk0, nchunks;      // this cavity's reduction chunks (runs of tiles)
  int32_t has_override;         // any finite sigma_override entry
  int32_t walls_only;           // no periodic face: every link either stays inside or hits a wall
  uint64_t div_nx_m, div_nxy_m; // magic multipliers: q = (i * m) >> s
  uint32_t div_nx_s, div_nxy_s;
  int64_t off;                  // byte offset of the cavity inside a state region
  int64_t plane;                // elements between population planes
  int64_t cell_off;             // first cell of the cavity in batch-wide cell arrays
  const double* tw;             // this cavity's wall-temperature fields (6 faces)
  int64_t twface[6];            // offset of each face inside tw
  // thermal
  double omega_T, cp_s, cp_l, cp_ref, lam_s, lam_l, latent, T_m, rho0;
  double hs, hl, inv_dh, inv_cps, inv_cpl, inv_rcw;  // inv_rcw = 1/(rho0 cp_ref omega_T)
  double sig_ovr[7];            // NaN: default rate
  // flow
  double s_nu, s_e, s_eps, s_q, s_pi, s_t, g_beta_rho0, T_ref;
  double fshift;                // rho0 for shifted storage, 0 for raw FP64
  double gshift;                // stored g_1..6 = g_a - gshift (16-bit formats; 0 otherwise)
  Pars<float> pf;               // the constants above in FP32
  Pars<double> pd;              // and in FP64
};

template <class R> __host__ __device__ inline const Pars<R>& pars(const CavParams& c);
template <> __host__ __device__ inline const Pars<float>& pars<float>(const CavParams& c) { return c.pf; }
template <> __host__ __device__ inline const Pars<double>& pars<double>(const CavParams& c) { return c.pd; }

// Device-side budget record of one cavity.
struct alignas(16) BudgetRec {
  double H, mass, fl;           // pre-collision sums of the last reduced step
  double flux_last, flux_cum;   // wall enthalpy inflow: last step, since creation
  double steps;                 // steps reduced so far
  double now_H, now_mass, now_fl;  // sums of the current state (measure pass)
  double now_flux0;             // inflow through the x- face in the next step
  double pad[2];
};

// Budget partials are written per wavefront (64 cells), without a workgroup
// barrier, so the waves of a tile retire independently.  Every step with
// partials writes its wall inflow into a dense per-wavefront array of its ring
// slot; full-partials steps also write the NPART state sums (h, rho, f_l,
// inflow, bad cells) of the wave into one shared record array, of which a
// reduction uses the last.  The measure pass writes the same records.
constexpr int NPART = 5;

// Accelerator complex dies of an MI355X.  The dispatcher hands workgroups to
// the XCDs round robin: workgroup b runs on XCD b mod kXcds.
constexpr int kXcds = 8;

struct StepArgs {
  const CavParams* cavs;
  const int2* tiles;            // (cavity, first cell) per tile
  int ntiles;
  const char* src;              // state region read (pre-collision state at t)
  char* dst;                    // state region written (pre-collision state at t+1)
  double* partials;             // wall inflow, one double per wavefront (budget >= 1)
  double* sums;                 // NPART doubles per wavefront (budget 2)
  const int32_t* status;        // per-cavity freeze flags
  int budget;                   // 0 none, 1 wall inflow only, 2 all partials
  int block, grid;              // grid = 0: one workgroup per tile
  int reverse;                  // 1: walk each XCD's queue positions from their end
  int flow, mrt;
  hipStream_t stream;
};

struct AdjArgs {
  const CavParams* cavs;
  const int2* tiles;
  int ntiles;
  const char* state;            // state at t (storage format)
  const char* lam_in;           // S^T lambda_{t+1}, stored by the step before (compute format)
  char* lam_out;                // S^T lambda_t (lambda_0 itself when last)
  double* dTw;                  // wall-temperature gradient accumulators (per cavity block)
  int block;
  int reverse;                  // 1: walk each XCD's queue positions from their end
  int last;                     // 1: the step to time 0 (stores lambda_0 itself, no dT_w terms)
  int flow, mrt;
  hipStream_t stream;
};

template <int P> hipError_t launch_step(const StepArgs& a);
template <int P> hipError_t launch_init(const CavParams* cavs, const int2* tiles, int ntiles,
                                        int block, int flow, char* dst, const double* T0,
                                        hipStream_t st);
template <int P> hipError_t launch_measure(const CavParams* cavs, const int2* tiles, int ntiles,
                                           int block, int flow, int mrt, const char* src,
                                           double* partials, hipStream_t st);
// single-cavity launchers: cav is a device pointer into the parameter table
template <int P> hipError_t launch_fields(const CavParams* cav, int64_t n, int flow,
                                          const char* src, uint32_t mask, double* out,
                                          hipStream_t st);
template <int P> hipError_t launch_get_state(const CavParams* cav, int64_t n, int flow,
                                             const char* src, double* f, double* g,
                                             hipStream_t st);
template <int P> hipError_t launch_set_state(const CavParams* cav, int64_t n, int flow,
                                             char* dst, const double* f, const double* g,
                                             hipStream_t st);
template <int P> hipError_t launch_adjoint(const AdjArgs& a);
template <int P> hipError_t launch_adj_seed(const CavParams* cav, int64_t n, int flow,
                                            double scale, const char* state, char* lam,
                                            double* dTw, hipStream_t st);
template <int P> hipError_t launch_adj_T0(const CavParams* cav, int64_t n, int flow,
                                          const char* state0, const char* lam, double* out,
                                          hipStream_t st);


}  // namespace lbpc

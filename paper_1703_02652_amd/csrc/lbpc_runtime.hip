// Runtime behind the lbpc C ABI: validation, workspace layout, tile queue,
// HIP graphs, budgets, launch-shape autotuning, checkpoints and the
// checkpointed discrete adjoint.  All device memory comes from the caller.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbpc.h"
#include "lbpc_api.hpp"

using namespace lbpc;

namespace {

constexpr int kRing = 16;           // budget partial slots (steps between reductions)
constexpr int kMinTile = 64;        // smallest tile: one wavefront
constexpr int kMaxTile = 256;       // largest tile: __launch_bounds__ of the kernels
constexpr int kChunk = 256;         // tiles per first-pass reduction workgroup
constexpr int kMaxRun = 1 << 24;    // longest XCD run of tiles
// Cells added to every population plane: keeps the planes of a cavity from
// starting at power-of-two distances (2^21 or 2^24 cells for 128^3 / 256^3),
// where the 26 concurrent plane streams fall on the same HBM channels.
constexpr int64_t kPlanePad = 256;
constexpr size_t kAlign = 256;
constexpr int kBudgetValues = 7;    // values per cavity returned by lbpc_budgets

size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

thread_local std::string g_err;

// ---------------------------------------------------------------------------
// Kernels that do not depend on the storage format
// ---------------------------------------------------------------------------
// Budget reduction, pass 1: one workgroup per (chunk, slot) sums the wavefront
// partials of a run of at most kChunk tiles of one cavity in a fixed order
// (wpt wavefronts per tile).  Steps (flux != null): the wall inflow of slot s
// from its dense array, the other sums from the shared records, for the last
// slot only (the step that wrote them).  Measure pass (flux == null): all
// NPART sums from the records.
__global__ void __launch_bounds__(256)
k_reduce_chunks(const int4* __restrict__ chunks, const double* __restrict__ flux,
                int64_t flux_stride, const double* __restrict__ sums, double* __restrict__ csum,
                int64_t csum_stride, int wpt) {
  __shared__ double sh[256][NPART];
  const int4 ch = chunks[blockIdx.x];  // (cavity, first tile, end tile, -)
  const bool last = blockIdx.y + 1 == gridDim.y;
  double v[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int w0 = ch.y * wpt, w1 = ch.z * wpt;
  for (int w = w0 + static_cast<int>(threadIdx.x); w < w1; w += blockDim.x) {
    if (flux) v[3] += flux[static_cast<int64_t>(blockIdx.y) * flux_stride + w];
    if (last) {
      const double* rec = sums + static_cast<int64_t>(w) * NPART;
      v[0] += rec[0];
      v[1] += rec[1];
      v[2] += rec[2];
      v[4] += rec[4];
      if (!flux) v[3] += rec[3];
    }
  }
#pragma unroll
  for (int k = 0; k < NPART; ++k) sh[threadIdx.x][k] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
#pragma unroll
      for (int k = 0; k < NPART; ++k) sh[threadIdx.x][k] += sh[threadIdx.x + w][k];
    }
    __syncthreads();
  }
  if (threadIdx.x < NPART)
    csum[static_cast<int64_t>(blockIdx.y) * csum_stride +
         static_cast<int64_t>(blockIdx.x) * NPART + threadIdx.x] = sh[0][threadIdx.x];
}

__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Pass 2: one workgroup per cavity; wavefront s sums the chunk sums of slot s
// (the same per-lane order as a single wavefront walking the slots), then one
// thread folds the slots in slot order.  mode 0 (steps): the wall inflow of
// every slot accumulates and the other sums are those of the last slot (the
// step that wrote full partials); mode 1 (measure of the current state): sums
// go to the now_* fields.
__global__ void __launch_bounds__(64 * kRing)
k_reduce_final(const CavParams* __restrict__ cavs, const double* __restrict__ csum,
               int64_t csum_stride, int nslots, int mode, BudgetRec* __restrict__ rec,
               int32_t* __restrict__ status) {
  __shared__ double tot[kRing][NPART];
  const CavParams& c = cavs[blockIdx.x];
  BudgetRec& r = rec[blockIdx.x];
  const int lane = threadIdx.x & 63, s = threadIdx.x >> 6;
  if (s < nslots) {
    double v[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = lane; j < c.nchunks; j += 64) {
#pragma unroll
      for (int k = 0; k < NPART; ++k)
        v[k] += csum[static_cast<int64_t>(s) * csum_stride + static_cast<int64_t>(c.chunk0 + j) * NPART + k];
    }
#pragma unroll
    for (int k = 0; k < NPART; ++k) v[k] = wave_total(v[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < NPART; ++k) tot[s][k] = v[k];
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double cum = r.flux_cum, last[NPART];
  for (int t = 0; t < nslots; ++t) cum += tot[t][3];
#pragma unroll
  for (int k = 0; k < NPART; ++k) last[k] = tot[nslots - 1][k];
  if (mode == 0) {
    r.H = last[0];
    r.mass = last[1];
    r.fl = last[2];
    r.flux_last = last[3];
    r.flux_cum = cum;
    r.steps += nslots;
  } else {
    r.now_H = last[0];
    r.now_mass = last[1];
    r.now_fl = last[2];
    r.now_flux0 = last[3];
  }
  if (last[4] > 0.0 || !isfinite(last[0]) || !isfinite(last[1]) || !isfinite(cum))
    status[blockIdx.x] = 1;
}

__global__ void __launch_bounds__(256) k_fill_zero(uint32_t* p, int64_t nwords) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < nwords;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of lbpc_budgets_noalloc: the chunk sums of its reductions
// (up to kRing slots) and the per-wavefront records of its measure pass.  One
// copy per device, held until the process ends; host code addresses it only
// through the device address that hipGetSymbolAddress returns for the current
// device (the array's name is a host-side stand-in).
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_address(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Layout
// ---------------------------------------------------------------------------
struct Layout {
  int batch = 0, prec = 0, flow = 0, mrt = 0;
  std::vector<int64_t> ncell, off, plane, cell_off, tw_off;
  std::vector<std::array<int64_t, 6>> twface;
  int64_t region_bytes = 0, total_cells = 0, max_tiles = 0, max_waves = 0, max_chunks = 0,
          tw_doubles = 0;
  size_t o_params = 0, o_tiles = 0, o_chunks = 0, o_csum = 0, o_tw = 0, o_status = 0, o_rec = 0,
         o_part = 0, o_sums = 0, o_mpart = 0, o_region0 = 0, o_region1 = 0, total = 0;
};

size_t pop_bytes(int prec) { return prec == 0 ? 8 : prec == 1 ? 4 : 2; }
// g_0: FP64; FP32 + an int16 correction in the FP32 format; FP32 in the 16-bit formats
size_t g0_bytes(int prec) { return prec == 0 ? 8 : prec == 1 ? 6 : 4; }

int64_t face_size(const lbpc_config& c, int face) {
  const int d = face / 2;
  if (d == 0) return static_cast<int64_t>(c.ny) * c.nz;
  if (d == 1) return static_cast<int64_t>(c.nx) * c.nz;
  return static_cast<int64_t>(c.nx) * c.ny;
}

bool validate(const lbpc_config* cfgs, int batch, std::string& err) {
  char buf[256];
  if (!cfgs || batch < 1) {
    err = "cfgs must hold at least one cavity";
    return false;
  }
  int64_t total = 0;
  for (int i = 0; i < batch; ++i) {
    const lbpc_config& c = cfgs[i];
    auto bad = [&](const char* what) {
      std::snprintf(buf, sizeof(buf), "cavity %d: %s", i, what);
      err = buf;
      return false;
    };
    if (c.nx < 1 || c.ny < 1 || c.nz < 1) return bad("nx, ny, nz must be >= 1");
    const int64_t n = static_cast<int64_t>(c.nx) * c.ny * c.nz;
    // kernels address a plane with 32-bit byte offsets of elements up to 8 bytes
    if (n + 128 + kPlanePad > (int64_t(1) << 29)) return bad("too many cells (limit 2^29 per cavity)");
    total += n;
    if (c.flow != 0 && c.flow != 1) return bad("flow must be 0 or 1");
    if (c.enth_model != LBPC_SRT && c.enth_model != LBPC_MRT) return bad("enth_model must be SRT or MRT");
    if (c.precision < 0 || c.precision > 3) return bad("unknown precision");
    if (c.precision != cfgs[0].precision || c.flow != cfgs[0].flow ||
        c.enth_model != cfgs[0].enth_model)
      return bad("precision, flow and enth_model must be the same for the whole batch");
    for (int f = 0; f < 6; ++f) {
      if (c.face_bc[f] < 0 || c.face_bc[f] > 2) return bad("unknown face boundary type");
      if (!std::isfinite(c.face_T[f])) return bad("face_T must be finite");
    }
    for (int d = 0; d < 3; ++d)
      if ((c.face_bc[2 * d] == LBPC_PERIODIC) != (c.face_bc[2 * d + 1] == LBPC_PERIODIC))
        return bad("a periodic face needs a periodic partner");
    if (!(c.omega_T > 0.0 && c.omega_T <= 1.0 / 3.0)) return bad("omega_T must lie in (0, 1/3]");
    if (!(c.cp_s > 0 && c.cp_l > 0 && c.cp_ref > 0)) return bad("specific heats must be > 0");
    if (!(c.lambda_s > 0 && c.lambda_l > 0)) return bad("conductivities must be > 0");
    if (!(c.rho0 > 0)) return bad("rho0 must be > 0");
    if (!std::isfinite(c.T_m) || !std::isfinite(c.T_ref) || !std::isfinite(c.g_beta) ||
        !std::isfinite(c.T_shift))
      return bad("T_m, T_ref, T_shift and g_beta must be finite");
    if (!(c.cp_l * c.T_m + c.latent > c.cp_s * c.T_m)) return bad("h_l must exceed h_s");
    if (c.flow) {
      if (!(c.nu > 0)) return bad("nu must be > 0");
      const double r[5] = {c.s_e, c.s_eps, c.s_q, c.s_pi, c.s_t};
      for (double v : r)
        if (!(v > 0.0 && v < 2.0)) return bad("flow relaxation rates must lie in (0, 2)");
    }
    for (int k = 0; k < 7; ++k) {
      const double v = c.sigma_override[k];
      if (!std::isnan(v) && !(v > 0.0 && v < 2.0)) return bad("sigma_override entries must be NaN or in (0, 2)");
    }
  }
  if (total >= (int64_t(1) << 31)) {
    err = "too many cells in the batch";
    return false;
  }
  return true;
}

Layout make_layout(const lbpc_config* cfgs, int batch) {
  Layout L;
  L.batch = batch;
  L.prec = cfgs[0].precision;
  L.flow = cfgs[0].flow;
  L.mrt = cfgs[0].enth_model;
  const size_t pb = pop_bytes(L.prec), g0b = g0_bytes(L.prec);
  int64_t off = 0, cells = 0, tiles = 0, chunks = 0, tw = 0, waves = 0;
  for (int i = 0; i < batch; ++i) {
    const lbpc_config& c = cfgs[i];
    const int64_t n = static_cast<int64_t>(c.nx) * c.ny * c.nz;
    const int64_t plane = (n + 127) / 128 * 128 + kPlanePad;
    L.ncell.push_back(n);
    L.plane.push_back(plane);
    L.off.push_back(off);
    L.cell_off.push_back(cells);
    const size_t bytes = static_cast<size_t>(plane) * ((L.flow ? 19 : 0) + 6) * pb +
                         static_cast<size_t>(plane) * g0b;
    off += static_cast<int64_t>(align_up(bytes));
    cells += n;
    const int64_t ct = (n + kMinTile - 1) / kMinTile;
    tiles += ct;
    chunks += (ct + kChunk - 1) / kChunk;
    // wavefronts of the tile queue for the tile size that needs the most of
    // them (the empty tail waves of the last tile write zero partials too)
    int64_t w = 0;
    for (int64_t b = kMinTile; b <= kMaxTile; b += kMinTile) w = std::max(w, (n + b - 1) / b * (b / 64));
    waves += w;
    std::array<int64_t, 6> tf;
    int64_t fo = 0;
    for (int f = 0; f < 6; ++f) {
      tf[f] = fo;
      fo += face_size(c, f);
    }
    L.twface.push_back(tf);
    L.tw_off.push_back(tw);
    tw += fo;
  }
  L.region_bytes = off;
  L.total_cells = cells;
  L.max_tiles = tiles;
  L.max_waves = waves;
  L.max_chunks = chunks;
  L.tw_doubles = tw;
  size_t o = 0;
  L.o_params = o; o = align_up(o + sizeof(CavParams) * batch);
  L.o_tiles = o; o = align_up(o + sizeof(int2) * tiles);
  L.o_chunks = o; o = align_up(o + sizeof(int4) * chunks);
  L.o_csum = o; o = align_up(o + sizeof(double) * NPART * chunks * kRing);
  L.o_tw = o; o = align_up(o + sizeof(double) * tw);
  L.o_status = o; o = align_up(o + sizeof(int32_t) * batch);
  L.o_rec = o; o = align_up(o + sizeof(BudgetRec) * batch);
  L.o_part = o; o = align_up(o + sizeof(double) * waves * kRing);
  L.o_sums = o; o = align_up(o + sizeof(double) * NPART * waves);
  L.o_mpart = o; o = align_up(o + sizeof(double) * NPART * waves);
  L.o_region0 = o; o = align_up(o + L.region_bytes);
  L.o_region1 = o; o = align_up(o + L.region_bytes);
  L.total = o;
  return L;
}

// Multiplier and shift for q = (i * m) >> s == i / d, exact for i < 2^31:
// m = floor(2^(32+l) / d) + 1 with l = ceil(log2 d).
void magic(uint32_t d, uint64_t& m, uint32_t& s) {
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  m = (uint64_t(1) << (32 + l)) / d + 1;
  s = 32 + l;
}

template <class R> void fill_pars(const CavParams& p, Pars<R>& q) {
  q.fshift = static_cast<R>(p.fshift);
  q.g_beta_rho0 = static_cast<R>(p.g_beta_rho0);
  q.T_ref = static_cast<R>(p.T_ref);
  q.s_nu = static_cast<R>(p.s_nu);
  q.s_e = static_cast<R>(p.s_e);
  q.s_eps = static_cast<R>(p.s_eps);
  q.s_q = static_cast<R>(p.s_q);
  q.s_pi = static_cast<R>(p.s_pi);
  q.s_t = static_cast<R>(p.s_t);
  q.lam_s = static_cast<R>(p.lam_s);
  q.dlam = static_cast<R>(p.lam_l - p.lam_s);
  q.inv_rcw = static_cast<R>(p.inv_rcw);
  q.cp_s = static_cast<R>(p.cp_s);
  q.dcp = static_cast<R>(p.cp_l - p.cp_s);
  q.w3 = static_cast<R>(3.0 * p.omega_T * p.cp_ref);
  q.w21 = static_cast<R>(21.0 * p.omega_T * p.cp_ref);
  q.whalf = static_cast<R>(0.5 * p.omega_T * p.cp_ref);
  q.wabb = static_cast<R>(p.omega_T * p.cp_ref);
  q.gshift = static_cast<R>(p.gshift);
  for (int k = 0; k < 7; ++k) q.sig_ovr[k] = static_cast<R>(p.sig_ovr[k]);
}

CavParams make_params(const lbpc_config& c, const Layout& L, int i, const double* d_tw) {
  CavParams p;
  std::memset(&p, 0, sizeof(p));
  p.nx = c.nx;
  p.ny = c.ny;
  p.nz = c.nz;
  p.n = static_cast<int32_t>(L.ncell[i]);
  p.nxy = c.nx * c.ny;
  p.walls_only = 1;
  for (int f = 0; f < 6; ++f) {
    p.bc[f] = c.face_bc[f];
    if (c.face_bc[f] == LBPC_PERIODIC) p.walls_only = 0;
  }
  magic(static_cast<uint32_t>(c.nx), p.div_nx_m, p.div_nx_s);
  magic(static_cast<uint32_t>(p.nxy), p.div_nxy_m, p.div_nxy_s);
  p.off = L.off[i];
  p.plane = L.plane[i];
  p.cell_off = L.cell_off[i];
  p.tw = d_tw + L.tw_off[i];
  for (int f = 0; f < 6; ++f) p.twface[f] = L.twface[i][f];
  p.omega_T = c.omega_T;
  p.cp_s = c.cp_s;
  p.cp_l = c.cp_l;
  p.cp_ref = c.cp_ref;
  p.lam_s = c.lambda_s;
  p.lam_l = c.lambda_l;
  p.latent = c.latent;
  p.T_m = c.T_m;
  p.rho0 = c.rho0;
  p.hs = c.cp_s * c.T_m;
  p.hl = c.cp_l * c.T_m + c.latent;
  p.inv_dh = 1.0 / (p.hl - p.hs);
  p.inv_cps = 1.0 / c.cp_s;
  p.inv_cpl = 1.0 / c.cp_l;
  p.inv_rcw = 1.0 / (c.rho0 * c.cp_ref * c.omega_T);
  p.has_override = 0;
  for (int k = 0; k < 7; ++k) {
    p.sig_ovr[k] = c.sigma_override[k];
    if (!std::isnan(c.sigma_override[k])) p.has_override = 1;
  }
  p.s_nu = 1.0 / (3.0 * c.nu + 0.5);  // Eq. (59)
  p.s_e = c.s_e;
  p.s_eps = c.s_eps;
  p.s_q = c.s_q;
  p.s_pi = c.s_pi;
  p.s_t = c.s_t;
  p.g_beta_rho0 = c.g_beta * c.rho0;
  p.T_ref = c.T_ref;
  p.fshift = c.precision == LBPC_FP64 ? 0.0 : c.rho0;
  p.gshift = c.precision >= LBPC_FP16S ? 0.5 * c.omega_T * c.cp_ref * c.T_shift : 0.0;
  fill_pars(p, p.pf);
  fill_pars(p, p.pd);
  return p;
}

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct AdjointPlan {
  bool ready = false;
  char* ws = nullptr;
  size_t bytes = 0;
  int64_t nsteps = 0, end_step = 0;
  int32_t every = 0, loss = 0;
  int nsnap = 0;
  bool last_seg_kept = false;  // the forward run left the last segment's states in place
  size_t o_snap = 0, o_seg = 0, o_lam0 = 0, o_lam1 = 0, o_dtw = 0, o_part = 0, total = 0;
  size_t lam_bytes = 0;
};

struct lbpc_ctx {
  Layout L;
  std::vector<lbpc_config> cfg;
  std::vector<CavParams> hp;
  std::vector<std::array<double, 6>> tw_mean;  // mean wall temperature of every face
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  char* ws = nullptr;
  CavParams* d_params = nullptr;
  int2* d_tiles = nullptr;
  int4* d_chunks = nullptr;
  double* d_csum = nullptr;
  double* d_tw = nullptr;
  int32_t* d_status = nullptr;
  BudgetRec* d_rec = nullptr;
  double* d_part = nullptr;   // wall inflow per wavefront, one array per ring slot
  double* d_sums = nullptr;   // state sums per wavefront (full-partials steps)
  double* d_mpart = nullptr;  // measure pass records
  char* region[2] = {nullptr, nullptr};
  char* scratch = nullptr;      // device address of the static scratch on this context's device
  int cur = 0;
  int flip = 0;                 // direction of the next step's walk of the queue
  int block = 256, grid = 0, graph_steps = 16, xrun = 4;
  int ntiles = 0, nchunks = 0;
  int pending = 0;
  int64_t steps = 0;
  bool unstable = false;
  // captured graphs of 1 to kRing steps from either state region
  hipGraphExec_t gexec[2][kRing + 1] = {};
  hipGraph_t graph[2][kRing + 1] = {};
  std::string err;
  AdjointPlan adj;
};

namespace {

int fail(lbpc_ctx* x, int code, const std::string& msg) {
  if (x) x->err = msg;
  g_err = msg;
  return code;
}

#define HIPCHK(x, call)                                                                 \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((x), LBPC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

hipError_t dispatch_step(lbpc_ctx* x, const char* src, char* dst, double* partials, int budget,
                         hipStream_t st) {
  StepArgs a;
  a.sums = x->d_sums;
  a.cavs = x->d_params;
  a.tiles = x->d_tiles;
  a.ntiles = x->ntiles;
  a.src = src;
  a.dst = dst;
  a.partials = partials;
  a.status = x->d_status;
  a.budget = budget;
  // consecutive steps walk the tile queue in opposite directions (a captured
  // graph starts forward and alternates from there; see capture)
  a.reverse = x->flip;
  x->flip ^= 1;
  a.block = x->block;
  a.grid = x->grid;
  a.flow = x->L.flow;
  a.mrt = x->L.mrt;
  a.stream = st;
  switch (x->L.prec) {
    case 0: return launch_step<0>(a);
    case 1: return launch_step<1>(a);
    case 2: return launch_step<2>(a);
    default: return launch_step<3>(a);
  }
}

hipError_t dispatch_measure(lbpc_ctx* x, const char* src, double* partials) {
  switch (x->L.prec) {
    case 0: return launch_measure<0>(x->d_params, x->d_tiles, x->ntiles, x->block, x->L.flow, x->L.mrt, src, partials, x->stream);
    case 1: return launch_measure<1>(x->d_params, x->d_tiles, x->ntiles, x->block, x->L.flow, x->L.mrt, src, partials, x->stream);
    case 2: return launch_measure<2>(x->d_params, x->d_tiles, x->ntiles, x->block, x->L.flow, x->L.mrt, src, partials, x->stream);
    default: return launch_measure<3>(x->d_params, x->d_tiles, x->ntiles, x->block, x->L.flow, x->L.mrt, src, partials, x->stream);
  }
}

hipError_t fill_zero(void* p, size_t bytes, hipStream_t st) {
  const int64_t words = static_cast<int64_t>(bytes / 4);
  if (words == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                     static_cast<uint32_t*>(p), words);
  return hipGetLastError();
}

// mode 0: the steps of the ring (inflow arrays from `partials`, state sums of
// the last one); mode 1: the measure pass (its records in `partials`).
// csum: chunk sums of up to kRing slots (the workspace's, or the static
// scratch of lbpc_budgets_noalloc).
hipError_t reduce(lbpc_ctx* x, const double* partials, int nslots, int mode, hipStream_t st,
                  double* csum = nullptr) {
  const int64_t csum_stride = x->L.max_chunks * NPART;
  if (!csum) csum = x->d_csum;
  const double* flux = mode == 0 ? partials : nullptr;
  const double* sums = mode == 0 ? x->d_sums : partials;
  hipLaunchKernelGGL(k_reduce_chunks, dim3(x->nchunks, nslots), dim3(256), 0, st, x->d_chunks,
                     flux, static_cast<int64_t>(x->L.max_waves), sums, csum, csum_stride,
                     x->block / 64);
  hipLaunchKernelGGL(k_reduce_final, dim3(x->L.batch), dim3(64 * nslots), 0, st, x->d_params,
                     csum, csum_stride, nslots, mode, x->d_rec, x->d_status);
  return hipGetLastError();
}

void drop_graphs(lbpc_ctx* x) {
  for (int i = 0; i < 2; ++i)
    for (int k = 0; k <= kRing; ++k) {
      // release paths have no caller to report a failure to
      if (x->gexec[i][k]) (void)hipGraphExecDestroy(x->gexec[i][k]);
      if (x->graph[i][k]) (void)hipGraphDestroy(x->graph[i][k]);
      x->gexec[i][k] = nullptr;
      x->graph[i][k] = nullptr;
    }
}

// Queue order for XCD runs of `run` tiles.  Queue position p = kXcds j + k
// runs on XCD k; it gets the j-th tile of that XCD, which walks the runs k,
// k + kXcds, k + 2 kXcds, ... of `run` consecutive tiles (in the natural order
// of the cells).  The tiles of one run are the rows on both sides of the
// diagonal links that cross between them: written from one XCD, the cache
// lines that both rows write are completed in that XCD's L2 before they go to
// memory.  Eight runs side by side keep the HBM streams sequential.  run = 1
// is the natural order; runs longer than a kXcds-th of the queue are cut to
// that length (one contiguous run per XCD).
std::vector<int2> xcd_order(const std::vector<int2>& tiles, int64_t run) {
  const int64_t m = static_cast<int64_t>(tiles.size());
  run = std::min<int64_t>(run, (m + kXcds - 1) / kXcds);
  if (run <= 1) return tiles;
  std::vector<int2> q;
  q.reserve(tiles.size());
  const int64_t runs = (m + run - 1) / run;
  const int64_t per_xcd = (runs + kXcds - 1) / kXcds;
  for (int64_t j = 0; j < per_xcd * run; ++j)
    for (int k = 0; k < kXcds; ++k) {
      const int64_t t = (k + kXcds * (j / run)) * run + j % run;
      if (t < m) q.push_back(tiles[t]);
    }
  return q;
}

// Queue order with one y-block per XCD: XCD k takes the tiles whose first row
// lies in the k-th eighth of the y range, slab after slab, so that the rows on
// both sides of every y- or z-crossing link are written from one XCD, a few
// dozen tiles apart.  Queue position kXcds j + k again holds XCD k's j-th tile.
std::vector<int2> yblock_order(const std::vector<int2>& tiles, const std::vector<lbpc_config>& cfg) {
  std::vector<std::vector<int2>> seq(kXcds);
  for (const int2& t : tiles) {
    const lbpc_config& c = cfg[static_cast<size_t>(t.x)];
    const int64_t y = (t.y / c.nx) % c.ny;
    seq[static_cast<size_t>(y * kXcds / c.ny)].push_back(t);
  }
  size_t longest = 0;
  for (const auto& v : seq) longest = std::max(longest, v.size());
  std::vector<int2> q;
  q.reserve(tiles.size());
  for (size_t j = 0; j < longest; ++j)
    for (int k = 0; k < kXcds; ++k)
      if (j < seq[static_cast<size_t>(k)].size()) q.push_back(seq[static_cast<size_t>(k)][j]);
  return q;
}

// Tile queue for the current block size (tiles never straddle cavities) in
// the XCD order; chunks and budget partials use the natural tile index.  The
// natural order takes the cavities largest first (stable for equal sizes):
// on the uneven 64-cavity batch (32^3 to 96^3) the step ran 2.7 % faster than
// in the order given, and a single cavity is unaffected.
int build_tiles(lbpc_ctx* x) {
  std::vector<int2> tiles;
  std::vector<int4> chunks;
  std::vector<int> order(static_cast<size_t>(x->L.batch));
  for (int i = 0; i < x->L.batch; ++i) order[static_cast<size_t>(i)] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return x->L.ncell[a] > x->L.ncell[b]; });
  for (int i : order) {
    x->hp[i].tile0 = static_cast<int32_t>(tiles.size());
    const int64_t n = x->L.ncell[i];
    for (int64_t c0 = 0; c0 < n; c0 += x->block) tiles.push_back(make_int2(i, static_cast<int>(c0)));
    x->hp[i].ntiles = static_cast<int32_t>(tiles.size()) - x->hp[i].tile0;
    x->hp[i].chunk0 = static_cast<int32_t>(chunks.size());
    for (int t = 0; t < x->hp[i].ntiles; t += kChunk)
      chunks.push_back(make_int4(i, x->hp[i].tile0 + t,
                                 x->hp[i].tile0 + std::min(t + kChunk, x->hp[i].ntiles), 0));
    x->hp[i].nchunks = static_cast<int32_t>(chunks.size()) - x->hp[i].chunk0;
  }
  x->ntiles = static_cast<int>(tiles.size());
  x->nchunks = static_cast<int>(chunks.size());
  // every wavefront of the queue owns one slot of each partial array
  if (static_cast<int64_t>(x->ntiles) * (x->block / 64) > x->L.max_waves ||
      x->nchunks > x->L.max_chunks || x->ntiles > x->L.max_tiles)
    return fail(x, LBPC_EINVAL, "tile queue larger than the workspace layout");
  tiles = x->xrun == 0 ? yblock_order(tiles, x->cfg) : xcd_order(tiles, x->xrun);
  HIPCHK(x, hipMemcpyAsync(x->d_tiles, tiles.data(), sizeof(int2) * tiles.size(),
                           hipMemcpyHostToDevice, x->stream));
  HIPCHK(x, hipMemcpyAsync(x->d_chunks, chunks.data(), sizeof(int4) * chunks.size(),
                           hipMemcpyHostToDevice, x->stream));
  HIPCHK(x, hipMemcpyAsync(x->d_params, x->hp.data(), sizeof(CavParams) * x->hp.size(),
                           hipMemcpyHostToDevice, x->stream));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  drop_graphs(x);
  return LBPC_OK;
}

int flush(lbpc_ctx* x, double* csum = nullptr) {
  if (x->pending > 0) {
    HIPCHK(x, reduce(x, x->d_part, x->pending, 0, x->stream, csum));
    x->pending = 0;
  }
  return LBPC_OK;
}

// One eager step: partials into the next ring slot, reduction when the ring fills.
int eager_step(lbpc_ctx* x) {
  double* part = x->d_part + static_cast<int64_t>(x->pending) * x->L.max_waves;
  HIPCHK(x, dispatch_step(x, x->region[x->cur], x->region[x->cur ^ 1], part, 2, x->stream));
  x->cur ^= 1;
  x->steps += 1;
  if (++x->pending == kRing) return flush(x);
  return LBPC_OK;
}

// Capture `count` steps plus their reduction, starting from region `from`.
// The graph's steps walk the queue forward, backward, ... from its first
// step on, whatever the host-side alternation is at capture time.
int capture(lbpc_ctx* x, int from, int count) {
  const int flip = x->flip;
  x->flip = 0;
  struct Restore {
    lbpc_ctx* x;
    int flip;
    ~Restore() { x->flip = flip; }
  } restore{x, flip};
  HIPCHK(x, hipStreamBeginCapture(x->cap, hipStreamCaptureModeThreadLocal));
  int c = from;
  hipError_t e = hipSuccess;
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    double* part = x->d_part + static_cast<int64_t>(i) * x->L.max_waves;
    e = dispatch_step(x, x->region[c], x->region[c ^ 1], part, i + 1 == count ? 2 : 1, x->cap);
    c ^= 1;
  }
  if (e == hipSuccess) e = reduce(x, x->d_part, count, 0, x->cap);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(x->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(x, LBPC_EHIP, std::string("graph capture: ") +
                                  hipGetErrorString(e != hipSuccess ? e : e2));
  }
  x->graph[from][count] = g;
  HIPCHK(x, hipGraphInstantiate(&x->gexec[from][count], g, nullptr, nullptr, 0));
  return LBPC_OK;
}

// Every graph a run can use (1 to graph_steps steps from either region),
// captured together the first time one is needed, so that capture and
// instantiation cost no time later in the run.
int ensure_graphs(lbpc_ctx* x) {
  for (int from = 0; from < 2; ++from)
    for (int count = 1; count <= x->graph_steps; ++count)
      if (!x->gexec[from][count]) {
        const int rc = capture(x, from, count);
        if (rc) return rc;
      }
  return LBPC_OK;
}

// Steps go into graphs of graph_steps steps, and the remainder into a graph
// of its own, each closed by its reduction; partials left by eager steps are
// reduced first, so every graph starts on an empty ring.  graph_steps = 0
// runs every step eagerly.
int run_steps(lbpc_ctx* x, int64_t n) {
  while (n > 0) {
    if (x->graph_steps > 0) {
      int rc = flush(x);
      if (rc) return rc;
      const int count = static_cast<int>(std::min<int64_t>(x->graph_steps, n));
      if (!x->gexec[x->cur][count]) {
        rc = ensure_graphs(x);
        if (rc) return rc;
      }
      HIPCHK(x, hipGraphLaunch(x->gexec[x->cur][count], x->stream));
      x->steps += count;
      x->cur ^= count & 1;
      x->flip = count & 1;  // the next step walks against the graph's last one
      n -= count;
    } else {
      const int rc = eager_step(x);
      if (rc) return rc;
      n -= 1;
    }
  }
  return LBPC_OK;
}

// A pair of timing events, destroyed on every exit path.
struct EventPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t create() {
    const hipError_t e = hipEventCreate(&e0);
    return e != hipSuccess ? e : hipEventCreate(&e1);
  }
  ~EventPair() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

int check_cavity(lbpc_ctx* x, int cavity) {
  if (!x) return fail(nullptr, LBPC_EINVAL, "null context");
  if (cavity < 0 || cavity >= x->L.batch) return fail(x, LBPC_EINVAL, "cavity index out of range");
  return LBPC_OK;
}

// Mean of a wall-temperature field (exactly the value of a uniform field).
double face_mean(const double* v, int64_t m) {
  double sum = 0.0;
  bool uniform = true;
  for (int64_t k = 0; k < m; ++k) {
    sum += v[k];
    uniform = uniform && v[k] == v[0];
  }
  return uniform ? v[0] : sum / static_cast<double>(m);
}

// Mean Nusselt number of the x- face, Eq. (65): Nu = -(l_c / dT) <dT/dx> on
// the wall with l_c = nx (hot-to-cold distance) and dT = <T_w> - T_m.  The
// wall gradient is the exact lattice heat flux of the anti-bounce-back links,
// q = -chi C_p,ref dT/dx per node and step, with chi = lambda_l / (rho0
// C_p,ref) of the liquid at the hot wall.  NaN when the face is not a
// fixed-temperature face or dT = 0.
double hot_wall_nusselt(const lbpc_config& c, double inflow, double tw_mean) {
  const double dT = tw_mean - c.T_m;
  if (c.face_bc[0] != LBPC_DIRICHLET || dT == 0.0) return std::nan("");
  const double q = inflow / (static_cast<double>(c.ny) * c.nz);
  const double chi = c.lambda_l / (c.rho0 * c.cp_ref);
  return q * c.nx / (chi * c.cp_ref * dT);
}

int read_status(lbpc_ctx* x, std::vector<int32_t>& st) {
  st.resize(x->L.batch);
  HIPCHK(x, hipMemcpyAsync(st.data(), x->d_status, sizeof(int32_t) * st.size(),
                           hipMemcpyDeviceToHost, x->stream));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  for (int32_t v : st)
    if (v) x->unstable = true;
  return LBPC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* lbpc_version(void) { return "lbpc 0.1 (gfx950)"; }

const char* lbpc_last_error(const lbpc_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_err.c_str();
}

size_t lbpc_workspace_bytes(const lbpc_config* cfgs, int32_t batch) {
  std::string err;
  if (!validate(cfgs, batch, err)) {
    g_err = err;
    return 0;
  }
  return make_layout(cfgs, batch).total;
}

int lbpc_create(const lbpc_config* cfgs, int32_t batch, void* dev_workspace, size_t bytes,
                const double* dev_T0, void* hip_stream, lbpc_ctx** out) {
  if (!out) return fail(nullptr, LBPC_EINVAL, "out must not be null");
  *out = nullptr;
  std::string err;
  if (!validate(cfgs, batch, err)) return fail(nullptr, LBPC_EINVAL, err);
  Layout L = make_layout(cfgs, batch);
  if (!dev_workspace) return fail(nullptr, LBPC_EINVAL, "workspace must not be null");
  if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign)
    return fail(nullptr, LBPC_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < L.total) return fail(nullptr, LBPC_ENOSPACE, "workspace too small");
  lbpc_ctx* x = new lbpc_ctx;
  x->L = L;
  x->cfg.assign(cfgs, cfgs + batch);
  x->stream = static_cast<hipStream_t>(hip_stream);
  x->ws = static_cast<char*>(dev_workspace);
  x->d_params = reinterpret_cast<CavParams*>(x->ws + L.o_params);
  x->d_tiles = reinterpret_cast<int2*>(x->ws + L.o_tiles);
  x->d_chunks = reinterpret_cast<int4*>(x->ws + L.o_chunks);
  x->d_csum = reinterpret_cast<double*>(x->ws + L.o_csum);
  x->d_tw = reinterpret_cast<double*>(x->ws + L.o_tw);
  x->d_status = reinterpret_cast<int32_t*>(x->ws + L.o_status);
  x->d_rec = reinterpret_cast<BudgetRec*>(x->ws + L.o_rec);
  x->d_part = reinterpret_cast<double*>(x->ws + L.o_part);
  x->d_sums = reinterpret_cast<double*>(x->ws + L.o_sums);
  x->d_mpart = reinterpret_cast<double*>(x->ws + L.o_mpart);
  x->region[0] = x->ws + L.o_region0;
  x->region[1] = x->ws + L.o_region1;
  for (int i = 0; i < batch; ++i) x->hp.push_back(make_params(cfgs[i], L, i, x->d_tw));
  auto cleanup = [&](int rc) {
    if (rc != LBPC_OK) {
      if (x->cap) (void)hipStreamDestroy(x->cap);
      delete x;
    }
    return rc;
  };
  if (hipStreamCreateWithFlags(&x->cap, hipStreamNonBlocking) != hipSuccess)
    return cleanup(fail(nullptr, LBPC_EHIP, "hipStreamCreate failed"));
  {
    const hipError_t e = scratch_address(&x->scratch);
    if (e != hipSuccess)
      return cleanup(fail(nullptr, LBPC_EHIP, std::string("static scratch address: ") +
                                                  hipGetErrorString(e)));
  }
  // wall fields start at the constant face temperatures
  std::vector<double> tw(static_cast<size_t>(L.tw_doubles));
  x->tw_mean.resize(batch);
  for (int i = 0; i < batch; ++i)
    for (int f = 0; f < 6; ++f) {
      const int64_t o = L.tw_off[i] + L.twface[i][f];
      std::fill(tw.begin() + o, tw.begin() + o + face_size(cfgs[i], f), cfgs[i].face_T[f]);
      x->tw_mean[i][f] = cfgs[i].face_T[f];
    }
  if (hipMemcpyAsync(x->d_tw, tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice,
                     x->stream) != hipSuccess ||
      fill_zero(x->d_status, sizeof(int32_t) * batch, x->stream) != hipSuccess ||
      fill_zero(x->d_rec, sizeof(BudgetRec) * batch, x->stream) != hipSuccess)
    return cleanup(fail(nullptr, LBPC_EHIP, "workspace initialisation failed"));
  int rc = build_tiles(x);
  if (rc) return cleanup(fail(nullptr, rc, x->err));
  hipError_t e;
  switch (L.prec) {
    case 0: e = launch_init<0>(x->d_params, x->d_tiles, x->ntiles, x->block, L.flow, x->region[0], dev_T0, x->stream); break;
    case 1: e = launch_init<1>(x->d_params, x->d_tiles, x->ntiles, x->block, L.flow, x->region[0], dev_T0, x->stream); break;
    case 2: e = launch_init<2>(x->d_params, x->d_tiles, x->ntiles, x->block, L.flow, x->region[0], dev_T0, x->stream); break;
    default: e = launch_init<3>(x->d_params, x->d_tiles, x->ntiles, x->block, L.flow, x->region[0], dev_T0, x->stream); break;
  }
  if (e != hipSuccess) return cleanup(fail(nullptr, LBPC_EHIP, hipGetErrorString(e)));
  if (hipStreamSynchronize(x->stream) != hipSuccess)
    return cleanup(fail(nullptr, LBPC_EHIP, "initialisation failed"));
  *out = x;
  return LBPC_OK;
}

void lbpc_destroy(lbpc_ctx* x) {
  if (!x) return;
  if (x->stream) (void)hipStreamSynchronize(x->stream);
  drop_graphs(x);
  if (x->cap) (void)hipStreamDestroy(x->cap);
  delete x;
}

int lbpc_set_wall_T(lbpc_ctx* x, int32_t cavity, int32_t face, const double* dev_Tw) {
  int rc = check_cavity(x, cavity);
  if (rc) return rc;
  if (face < 0 || face > 5 || !dev_Tw) return fail(x, LBPC_EINVAL, "bad face or null field");
  if (x->cfg[cavity].face_bc[face] != LBPC_DIRICHLET)
    return fail(x, LBPC_EINVAL, "face is not a fixed-temperature face");
  double* dst = x->d_tw + x->L.tw_off[cavity] + x->L.twface[cavity][face];
  const int64_t nodes = face_size(x->cfg[cavity], face);
  HIPCHK(x, hipMemcpyAsync(dst, dev_Tw, sizeof(double) * nodes, hipMemcpyDeviceToDevice,
                           x->stream));
  // the face mean enters the Nusselt number of lbpc_budgets
  std::vector<double> h(static_cast<size_t>(nodes));
  HIPCHK(x, hipMemcpyAsync(h.data(), dev_Tw, sizeof(double) * nodes, hipMemcpyDeviceToHost,
                           x->stream));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  x->tw_mean[cavity][face] = face_mean(h.data(), nodes);
  return LBPC_OK;
}

int lbpc_step(lbpc_ctx* x, int64_t nsteps) {
  if (!x) return fail(nullptr, LBPC_EINVAL, "null context");
  if (nsteps < 0) return fail(x, LBPC_EINVAL, "nsteps must be >= 0");
  if (x->unstable) return fail(x, LBPC_EUNSTABLE, "a cavity was flagged unstable");
  return run_steps(x, nsteps);
}

int lbpc_fields(lbpc_ctx* x, int32_t cavity, uint32_t mask, double* dev_out) {
  int rc = check_cavity(x, cavity);
  if (rc) return rc;
  if (!dev_out || mask == 0 || mask > 31) return fail(x, LBPC_EINVAL, "bad mask or null output");
  const CavParams* cp = x->d_params + cavity;
  const int64_t n = x->L.ncell[cavity];
  hipError_t e;
  switch (x->L.prec) {
    case 0: e = launch_fields<0>(cp, n, x->L.flow, x->region[x->cur], mask, dev_out, x->stream); break;
    case 1: e = launch_fields<1>(cp, n, x->L.flow, x->region[x->cur], mask, dev_out, x->stream); break;
    case 2: e = launch_fields<2>(cp, n, x->L.flow, x->region[x->cur], mask, dev_out, x->stream); break;
    default: e = launch_fields<3>(cp, n, x->L.flow, x->region[x->cur], mask, dev_out, x->stream); break;
  }
  HIPCHK(x, e);
  return LBPC_OK;
}

int lbpc_budgets(lbpc_ctx* x, double* host_out) {
  if (!x || !host_out) return fail(x, LBPC_EINVAL, "null argument");
  int rc = flush(x);
  if (rc) return rc;
  HIPCHK(x, dispatch_measure(x, x->region[x->cur], x->d_mpart));
  HIPCHK(x, reduce(x, x->d_mpart, 1, 1, x->stream));
  std::vector<BudgetRec> rec(x->L.batch);
  HIPCHK(x, hipMemcpyAsync(rec.data(), x->d_rec, sizeof(BudgetRec) * rec.size(),
                           hipMemcpyDeviceToHost, x->stream));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  for (int i = 0; i < x->L.batch; ++i) {
    double* o = host_out + kBudgetValues * i;
    o[0] = rec[i].now_H;
    o[1] = rec[i].now_mass;
    o[2] = rec[i].now_fl;
    o[3] = rec[i].flux_cum;
    o[4] = static_cast<double>(x->steps);
    o[5] = rec[i].now_flux0;
    o[6] = hot_wall_nusselt(x->cfg[i], rec[i].now_flux0, x->tw_mean[i][0]);
  }
  std::vector<int32_t> st;
  return read_status(x, st);
}

int lbpc_budgets_noalloc(lbpc_ctx* x, double* host_out) {
  if (!x || !host_out) return fail(x, LBPC_EINVAL, "null argument");
  // scratch: [chunk sums of kRing slots][measure records], 256-byte aligned
  const size_t csum_bytes =
      align_up(sizeof(double) * NPART * static_cast<size_t>(x->L.max_chunks) * kRing);
  const size_t rec_bytes = sizeof(double) * NPART * static_cast<size_t>(x->L.max_waves);
  if (csum_bytes + rec_bytes > kScratchBytes) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "lbpc_budgets_noalloc: this batch needs %zu bytes of scratch, more than the "
                  "%zu the library holds per device (use lbpc_budgets)",
                  csum_bytes + rec_bytes, kScratchBytes);
    return fail(x, LBPC_ENOSPACE, msg);
  }
  double* csum = reinterpret_cast<double*>(x->scratch);
  double* mrec = reinterpret_cast<double*>(x->scratch + csum_bytes);
  int rc = flush(x, csum);
  if (rc) return rc;
  HIPCHK(x, dispatch_measure(x, x->region[x->cur], mrec));
  HIPCHK(x, reduce(x, mrec, 1, 1, x->stream, csum));
  // records and status through fixed host buffers on the stack, a chunk at a time
  constexpr int kChunkCav = 32;
  BudgetRec rec[kChunkCav];
  int32_t st[kChunkCav];
  for (int i0 = 0; i0 < x->L.batch; i0 += kChunkCav) {
    const int m = std::min(kChunkCav, x->L.batch - i0);
    HIPCHK(x, hipMemcpyAsync(rec, x->d_rec + i0, sizeof(BudgetRec) * m, hipMemcpyDeviceToHost,
                             x->stream));
    HIPCHK(x, hipMemcpyAsync(st, x->d_status + i0, sizeof(int32_t) * m, hipMemcpyDeviceToHost,
                             x->stream));
    HIPCHK(x, hipStreamSynchronize(x->stream));
    for (int k = 0; k < m; ++k) {
      const int i = i0 + k;
      double* o = host_out + kBudgetValues * i;
      o[0] = rec[k].now_H;
      o[1] = rec[k].now_mass;
      o[2] = rec[k].now_fl;
      o[3] = rec[k].flux_cum;
      o[4] = static_cast<double>(x->steps);
      o[5] = rec[k].now_flux0;
      o[6] = hot_wall_nusselt(x->cfg[i], rec[k].now_flux0, x->tw_mean[i][0]);
      if (st[k]) x->unstable = true;
    }
  }
  return LBPC_OK;
}

int lbpc_status(lbpc_ctx* x, int32_t* host_flags) {
  if (!x || !host_flags) return fail(x, LBPC_EINVAL, "null argument");
  int rc = flush(x);
  if (rc) return rc;
  std::vector<int32_t> st;
  rc = read_status(x, st);
  if (rc) return rc;
  std::copy(st.begin(), st.end(), host_flags);
  return LBPC_OK;
}

int lbpc_get_state(lbpc_ctx* x, int32_t cavity, double* dev_f, double* dev_g) {
  int rc = check_cavity(x, cavity);
  if (rc) return rc;
  if (!dev_g || (x->L.flow && !dev_f)) return fail(x, LBPC_EINVAL, "null output");
  const CavParams* cp = x->d_params + cavity;
  const int64_t n = x->L.ncell[cavity];
  hipError_t e;
  switch (x->L.prec) {
    case 0: e = launch_get_state<0>(cp, n, x->L.flow, x->region[x->cur], dev_f, dev_g, x->stream); break;
    case 1: e = launch_get_state<1>(cp, n, x->L.flow, x->region[x->cur], dev_f, dev_g, x->stream); break;
    case 2: e = launch_get_state<2>(cp, n, x->L.flow, x->region[x->cur], dev_f, dev_g, x->stream); break;
    default: e = launch_get_state<3>(cp, n, x->L.flow, x->region[x->cur], dev_f, dev_g, x->stream); break;
  }
  HIPCHK(x, e);
  return LBPC_OK;
}

int lbpc_set_state(lbpc_ctx* x, int32_t cavity, const double* dev_f, const double* dev_g) {
  int rc = check_cavity(x, cavity);
  if (rc) return rc;
  if (!dev_g || (x->L.flow && !dev_f)) return fail(x, LBPC_EINVAL, "null input");
  const CavParams* cp = x->d_params + cavity;
  const int64_t n = x->L.ncell[cavity];
  hipError_t e;
  switch (x->L.prec) {
    case 0: e = launch_set_state<0>(cp, n, x->L.flow, x->region[x->cur], dev_f, dev_g, x->stream); break;
    case 1: e = launch_set_state<1>(cp, n, x->L.flow, x->region[x->cur], dev_f, dev_g, x->stream); break;
    case 2: e = launch_set_state<2>(cp, n, x->L.flow, x->region[x->cur], dev_f, dev_g, x->stream); break;
    default: e = launch_set_state<3>(cp, n, x->L.flow, x->region[x->cur], dev_f, dev_g, x->stream); break;
  }
  HIPCHK(x, e);
  x->adj.ready = false;
  return LBPC_OK;
}

// Checkpoint: header, the current state region, budget records, status, wall fields.
size_t lbpc_state_bytes(const lbpc_ctx* x) {
  if (!x) return 0;
  return 64 + static_cast<size_t>(x->L.region_bytes) + sizeof(BudgetRec) * x->L.batch +
         sizeof(int32_t) * x->L.batch + sizeof(double) * x->L.tw_doubles;
}

int lbpc_save(lbpc_ctx* x, void* host_buf, size_t bytes) {
  if (!x || !host_buf) return fail(x, LBPC_EINVAL, "null argument");
  if (bytes < lbpc_state_bytes(x)) return fail(x, LBPC_ENOSPACE, "buffer too small");
  int rc = flush(x);
  if (rc) return rc;
  char* p = static_cast<char*>(host_buf);
  int64_t hdr[8] = {0x6c627063, x->L.batch, x->L.region_bytes, x->steps, x->L.prec, x->L.flow,
                    x->L.tw_doubles, 0};
  std::memcpy(p, hdr, sizeof(hdr));
  p += 64;
  HIPCHK(x, hipMemcpyAsync(p, x->region[x->cur], x->L.region_bytes, hipMemcpyDeviceToHost, x->stream));
  p += x->L.region_bytes;
  HIPCHK(x, hipMemcpyAsync(p, x->d_rec, sizeof(BudgetRec) * x->L.batch, hipMemcpyDeviceToHost, x->stream));
  p += sizeof(BudgetRec) * x->L.batch;
  HIPCHK(x, hipMemcpyAsync(p, x->d_status, sizeof(int32_t) * x->L.batch, hipMemcpyDeviceToHost, x->stream));
  p += sizeof(int32_t) * x->L.batch;
  HIPCHK(x, hipMemcpyAsync(p, x->d_tw, sizeof(double) * x->L.tw_doubles, hipMemcpyDeviceToHost, x->stream));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  return LBPC_OK;
}

int lbpc_load(lbpc_ctx* x, const void* host_buf, size_t bytes) {
  if (!x || !host_buf) return fail(x, LBPC_EINVAL, "null argument");
  if (bytes < lbpc_state_bytes(x)) return fail(x, LBPC_ENOSPACE, "buffer too small");
  const char* p = static_cast<const char*>(host_buf);
  int64_t hdr[8];
  std::memcpy(hdr, p, sizeof(hdr));
  if (hdr[0] != 0x6c627063 || hdr[1] != x->L.batch || hdr[2] != x->L.region_bytes ||
      hdr[4] != x->L.prec || hdr[5] != x->L.flow || hdr[6] != x->L.tw_doubles)
    return fail(x, LBPC_EINVAL, "checkpoint does not match this context");
  int rc = flush(x);
  if (rc) return rc;
  p += 64;
  HIPCHK(x, hipMemcpyAsync(x->region[x->cur], p, x->L.region_bytes, hipMemcpyHostToDevice, x->stream));
  p += x->L.region_bytes;
  HIPCHK(x, hipMemcpyAsync(x->d_rec, p, sizeof(BudgetRec) * x->L.batch, hipMemcpyHostToDevice, x->stream));
  p += sizeof(BudgetRec) * x->L.batch;
  HIPCHK(x, hipMemcpyAsync(x->d_status, p, sizeof(int32_t) * x->L.batch, hipMemcpyHostToDevice, x->stream));
  p += sizeof(int32_t) * x->L.batch;
  HIPCHK(x, hipMemcpyAsync(x->d_tw, p, sizeof(double) * x->L.tw_doubles, hipMemcpyHostToDevice, x->stream));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  std::vector<double> tw(static_cast<size_t>(x->L.tw_doubles));
  std::memcpy(tw.data(), p, sizeof(double) * tw.size());
  for (int i = 0; i < x->L.batch; ++i)
    for (int f = 0; f < 6; ++f) {
      const int64_t o = x->L.tw_off[i] + x->L.twface[i][f];
      x->tw_mean[i][f] = face_mean(tw.data() + o, face_size(x->cfg[i], f));
    }
  x->steps = hdr[3];
  x->unstable = false;
  x->adj.ready = false;
  std::vector<int32_t> st;
  return read_status(x, st);
}

int lbpc_set_launch(lbpc_ctx* x, int32_t block, int32_t grid_blocks, int32_t graph_steps,
                    int32_t xcd_run) {
  if (!x) return fail(nullptr, LBPC_EINVAL, "null context");
  if (block < kMinTile || block > kMaxTile || block % 64)
    return fail(x, LBPC_EINVAL, "block must be 64, 128, 192 or 256");
  if (grid_blocks < 0) return fail(x, LBPC_EINVAL, "grid_blocks must be >= 0");
  if (graph_steps < 0 || graph_steps > kRing)
    return fail(x, LBPC_EINVAL, "graph_steps must lie in [0, 16]");
  if (xcd_run < 0 || xcd_run > kMaxRun) return fail(x, LBPC_EINVAL, "xcd_run must lie in [0, 2^24]");
  int rc = flush(x);
  if (rc) return rc;
  x->grid = grid_blocks;
  x->graph_steps = graph_steps;
  if (block != x->block || xcd_run != x->xrun) {
    x->block = block;
    x->xrun = xcd_run;
    rc = build_tiles(x);
    if (rc) return rc;
  }
  drop_graphs(x);
  return LBPC_OK;
}

int lbpc_get_launch(const lbpc_ctx* x, int32_t* block, int32_t* grid_blocks, int32_t* graph_steps,
                    int32_t* xcd_run) {
  if (!x) return LBPC_EINVAL;
  if (block) *block = x->block;
  if (grid_blocks) *grid_blocks = x->grid;
  if (graph_steps) *graph_steps = x->graph_steps;
  if (xcd_run) *xcd_run = x->xrun;
  return LBPC_OK;
}

int lbpc_time_step_kernel(lbpc_ctx* x, int32_t nsteps, double* host_ms_out) {
  if (!x || nsteps < 1) return fail(x, LBPC_EINVAL, "bad argument");
  int rc = flush(x);
  if (rc) return rc;
  // The step kernel as the run's graphs hold it: a captured graph of kTimed
  // back-to-back wall-inflow-partials steps, timed between one event pair per
  // replay.  Each replay is followed by two untimed eager steps, the second
  // with all partials, which close the ring and bring the state back to the
  // region the graph starts from.
  constexpr int kTimed = kRing - 2;
  struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    ~Graph() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
    }
  } tg;
  HIPCHK(x, hipStreamBeginCapture(x->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  int c = x->cur;
  for (int i = 0; i < kTimed && e == hipSuccess; ++i, c ^= 1)
    e = dispatch_step(x, x->region[c], x->region[c ^ 1],
                      x->d_part + static_cast<int64_t>(i) * x->L.max_waves, 1, x->cap);
  const hipError_t e2 = hipStreamEndCapture(x->cap, &tg.g);
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(x, LBPC_EHIP, std::string("timing graph capture: ") +
                                  hipGetErrorString(e != hipSuccess ? e : e2));
  HIPCHK(x, hipGraphInstantiate(&tg.e, tg.g, nullptr, nullptr, 0));
  EventPair ev;
  HIPCHK(x, ev.create());
  const int runs = (nsteps + kTimed - 1) / kTimed;
  double total = 0.0;
  for (int r = 0; r < runs; ++r) {
    HIPCHK(x, hipEventRecord(ev.e0, x->stream));
    HIPCHK(x, hipGraphLaunch(tg.e, x->stream));
    HIPCHK(x, hipEventRecord(ev.e1, x->stream));
    x->steps += kTimed;
    x->pending = kTimed;
    for (int budget = 1; budget <= 2; ++budget) {
      double* part = x->d_part + static_cast<int64_t>(x->pending) * x->L.max_waves;
      HIPCHK(x, dispatch_step(x, x->region[x->cur], x->region[x->cur ^ 1], part, budget,
                              x->stream));
      x->cur ^= 1;
      x->steps += 1;
      x->pending += 1;
    }
    rc = flush(x);
    if (rc) return rc;
    HIPCHK(x, hipEventSynchronize(ev.e1));
    float ms = 0.f;
    HIPCHK(x, hipEventElapsedTime(&ms, ev.e0, ev.e1));
    total += ms;
  }
  if (host_ms_out) *host_ms_out = total / (static_cast<double>(runs) * kTimed);
  return LBPC_OK;
}

int lbpc_autotune(lbpc_ctx* x, int32_t trial_steps, double* host_ms_out) {
  if (!x || trial_steps < 1) return fail(x, LBPC_EINVAL, "bad argument");
  int rc = flush(x);
  if (rc) return rc;
  hipDeviceProp_t prop;
  int dev = 0;
  HIPCHK(x, hipGetDevice(&dev));
  HIPCHK(x, hipGetDeviceProperties(&prop, dev));
  const int cus = prop.multiProcessorCount;
  const int blocks[3] = {64, 128, 256};
  const int grids[2] = {0, 4 * cus};
  // Trials run real, alternating steps (the cache state of a run differs from
  // re-reading one unchanged region); the state is saved to the host first and
  // restored afterwards, so tuning leaves the run untouched.
  std::vector<char> saved(static_cast<size_t>(x->L.region_bytes));
  const int cur0 = x->cur;
  HIPCHK(x, hipMemcpyAsync(saved.data(), x->region[cur0], saved.size(), hipMemcpyDeviceToHost,
                           x->stream));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  EventPair ev;
  HIPCHK(x, ev.create());
  struct Cand {
    int b, g, xc;
    double ms;
  };
  int c = cur0;
  // time `steps` steps of the configuration (after two unmeasured ones); the
  // trials run the step without budget partials, so that profiles of the run
  // that follows see only the chosen launch in the partials kernels
  auto trial = [&](const Cand& k, int steps, double& per) -> int {
    if (k.b != x->block || k.xc != x->xrun) {
      x->block = k.b;
      x->xrun = k.xc;
      const int r = build_tiles(x);
      if (r) return r;
    }
    x->grid = k.g;
    for (int i = 0; i < 2; ++i, c ^= 1)
      HIPCHK(x, dispatch_step(x, x->region[c], x->region[c ^ 1], nullptr, 0, x->stream));
    HIPCHK(x, hipEventRecord(ev.e0, x->stream));
    for (int i = 0; i < steps; ++i, c ^= 1)
      HIPCHK(x, dispatch_step(x, x->region[c], x->region[c ^ 1], nullptr, 0, x->stream));
    HIPCHK(x, hipEventRecord(ev.e1, x->stream));
    HIPCHK(x, hipEventSynchronize(ev.e1));
    float ms = 0.f;
    HIPCHK(x, hipEventElapsedTime(&ms, ev.e0, ev.e1));
    per = ms / steps;
    return LBPC_OK;
  };
  // stage 1: every shape once; stage 2: the three fastest again, interleaved,
  // four rounds each (a drift of the device clock then hits all three alike)
  Cand best{x->block, x->grid, x->xrun, 0.0};
  auto tune = [&]() -> int {
    std::vector<Cand> cands;
    for (int b : blocks) {
      int64_t ntiles = 0;
      for (int64_t n : x->L.ncell) ntiles += (n + b - 1) / b;
      // queue orders: one y-block per XCD (0), natural order (1), XCD runs of
      // 2 to 32 tiles, one contiguous run per XCD
      const int whole = static_cast<int>((ntiles + kXcds - 1) / kXcds);
      std::vector<int> runs = {0, 1, 2, 4, 8, 16, 32};
      if (whole > 32) runs.push_back(whole);
      for (int g : grids)
        for (int xc : runs) {
          // a persistent grid must have fewer workgroups than there are tiles
          if (g > 0 && g >= ntiles) continue;
          cands.push_back({b, g, xc, 0.0});
        }
    }
    for (Cand& k : cands) {
      const int r = trial(k, trial_steps, k.ms);
      if (r) return r;
    }
    std::sort(cands.begin(), cands.end(), [](const Cand& p, const Cand& q) { return p.ms < q.ms; });
    const size_t top = std::min<size_t>(3, cands.size());
    std::vector<double> sum(top, 0.0);
    for (int round = 0; round < 4; ++round)
      for (size_t i = 0; i < top; ++i) {
        double per = 0.0;
        const int r = trial(cands[i], trial_steps, per);
        if (r) return r;
        sum[i] += per;
      }
    size_t pick = 0;
    for (size_t i = 1; i < top; ++i)
      if (sum[i] < sum[pick]) pick = i;
    best = cands[pick];
    best.ms = sum[pick] / 4.0;
    return LBPC_OK;
  };
  // on failure the previous launch is kept; the state is restored either way
  const int trc = tune();
  const std::string terr = x->err;
  const hipError_t e1 = hipMemcpyAsync(x->region[cur0], saved.data(), saved.size(),
                                       hipMemcpyHostToDevice, x->stream);
  const hipError_t e2 = hipStreamSynchronize(x->stream);
  x->cur = cur0;
  x->block = best.b;
  x->grid = best.g;
  x->xrun = best.xc;
  rc = build_tiles(x);
  if (trc) return fail(x, trc, terr);
  if (e1 != hipSuccess || e2 != hipSuccess)
    return fail(x, LBPC_EHIP, std::string("restoring the state after tuning: ") +
                                  hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  if (rc) return rc;
  if (host_ms_out) *host_ms_out = best.ms;
  return LBPC_OK;
}

// ---------------------------------------------------------------------------
// Checkpointed discrete adjoint
// ---------------------------------------------------------------------------
static AdjointPlan plan_adjoint(const lbpc_ctx* x, int64_t nsteps, int32_t every) {
  AdjointPlan a;
  a.nsteps = nsteps;
  a.every = every;
  a.nsnap = static_cast<int>((nsteps + every - 1) / every);
  const size_t rb = static_cast<size_t>(x->L.region_bytes);
  const size_t rsz = x->L.prec == 0 ? 8 : 4;
  a.lam_bytes = align_up(static_cast<size_t>(x->L.plane[0]) * ((x->L.flow ? 19 : 0) + 7) * rsz);
  size_t o = 0;
  a.o_snap = o; o += rb * static_cast<size_t>(a.nsnap);
  a.o_seg = o; o += rb * static_cast<size_t>(std::max(every - 1, 0));
  a.o_lam0 = o; o += a.lam_bytes;
  a.o_lam1 = o; o += a.lam_bytes;
  a.o_dtw = o; o = align_up(o + sizeof(double) * x->L.tw_doubles);
  a.total = o;
  return a;
}

size_t lbpc_adjoint_workspace_bytes(const lbpc_ctx* x, int64_t nsteps, int32_t every) {
  if (!x || nsteps < 1 || every < 1) return 0;
  return plan_adjoint(x, nsteps, every).total;
}

int lbpc_adjoint_forward(lbpc_ctx* x, int64_t nsteps, int32_t every, int32_t loss,
                         void* dev_adj_ws, size_t bytes, double* host_loss) {
  if (!x) return fail(nullptr, LBPC_EINVAL, "null context");
  if (x->L.batch != 1) return fail(x, LBPC_EINVAL, "the adjoint needs a single-cavity context");
  if (x->L.prec > 1) return fail(x, LBPC_EINVAL, "the adjoint needs FP64 or FP32 storage");
  if (nsteps < 1 || every < 1 || (loss != 0 && loss != 1))
    return fail(x, LBPC_EINVAL, "bad nsteps, ckpt_every or loss");
  if (x->unstable) return fail(x, LBPC_EUNSTABLE, "a cavity was flagged unstable");
  AdjointPlan a = plan_adjoint(x, nsteps, every);
  if (!dev_adj_ws || reinterpret_cast<uintptr_t>(dev_adj_ws) % kAlign)
    return fail(x, LBPC_EINVAL, "adjoint workspace must be non-null and 256-byte aligned");
  if (bytes < a.total) return fail(x, LBPC_ENOSPACE, "adjoint workspace too small");
  a.ws = static_cast<char*>(dev_adj_ws);
  a.bytes = bytes;
  a.loss = loss;
  int rc = flush(x);
  if (rc) return rc;
  const size_t rb = static_cast<size_t>(x->L.region_bytes);
  if (every == 1) {
    // a snapshot of every state: each step writes straight into the next
    // snapshot slot (no copies; the backward sweep then recomputes nothing)
    char* snap = a.ws + a.o_snap;
    HIPCHK(x, hipMemcpyAsync(snap, x->region[x->cur], rb, hipMemcpyDeviceToDevice, x->stream));
    for (int64_t t = 0; t < nsteps; ++t) {
      char* dst = t + 1 < nsteps ? snap + rb * static_cast<size_t>(t + 1) : x->region[x->cur ^ 1];
      double* part = x->d_part + static_cast<int64_t>(x->pending) * x->L.max_waves;
      // all partials only where a reduction closes (as the graphs do)
      const int budget = (x->pending + 1 == kRing || t + 1 == nsteps) ? 2 : 1;
      HIPCHK(x, dispatch_step(x, snap + rb * static_cast<size_t>(t), dst, part, budget, x->stream));
      x->steps += 1;
      if (++x->pending == kRing) {
        rc = flush(x);
        if (rc) return rc;
      }
    }
    x->cur ^= 1;
  } else {
    for (int64_t s = 0; s < nsteps; s += every) {
      HIPCHK(x, hipMemcpyAsync(a.ws + a.o_snap + rb * static_cast<size_t>(s / every),
                               x->region[x->cur], rb, hipMemcpyDeviceToDevice, x->stream));
      const int64_t len = std::min<int64_t>(every, nsteps - s);
      if (s + len < nsteps) {
        rc = run_steps(x, len);
        if (rc) return rc;
        continue;
      }
      // the last segment writes its states straight into the recomputation
      // slots, so that the backward sweep starts without recomputing it
      char* seg = a.ws + a.o_seg;
      for (int64_t t = 0; t < len; ++t) {
        const char* src = t == 0 ? x->region[x->cur] : seg + rb * static_cast<size_t>(t - 1);
        char* dst = t + 1 < len ? seg + rb * static_cast<size_t>(t) : x->region[x->cur ^ 1];
        double* part = x->d_part + static_cast<int64_t>(x->pending) * x->L.max_waves;
        const int budget = (x->pending + 1 == kRing || t + 1 == len) ? 2 : 1;
        HIPCHK(x, dispatch_step(x, src, dst, part, budget, x->stream));
        x->steps += 1;
        if (++x->pending == kRing) {
          rc = flush(x);
          if (rc) return rc;
        }
      }
      x->cur ^= 1;
      a.last_seg_kept = true;
    }
  }
  a.end_step = x->steps;
  double b[6];
  rc = lbpc_budgets(x, b);
  if (rc) return rc;
  if (x->unstable) return fail(x, LBPC_EUNSTABLE, "the forward run became unstable");
  const double area = static_cast<double>(x->cfg[0].ny) * x->cfg[0].nz;
  if (host_loss) *host_loss = loss == 0 ? b[2] : b[2] / area;
  a.ready = true;
  x->adj = a;
  return LBPC_OK;
}

int lbpc_adjoint_backward(lbpc_ctx* x, double seed, double* dev_dL_dTw, double* dev_dL_dT0) {
  if (!x) return fail(nullptr, LBPC_EINVAL, "null context");
  AdjointPlan& a = x->adj;
  if (!a.ready || a.end_step != x->steps)
    return fail(x, LBPC_EINVAL, "no matching lbpc_adjoint_forward for the current state");
  int rc = flush(x);
  if (rc) return rc;
  const size_t rb = static_cast<size_t>(x->L.region_bytes);
  const int64_t n = x->L.ncell[0];
  const CavParams* cp = x->d_params;
  char* lam[2] = {a.ws + a.o_lam0, a.ws + a.o_lam1};
  double* dtw = reinterpret_cast<double*>(a.ws + a.o_dtw);
  HIPCHK(x, fill_zero(dtw, sizeof(double) * x->L.tw_doubles, x->stream));
  const double area = static_cast<double>(x->cfg[0].ny) * x->cfg[0].nz;
  const double scale = a.loss == 0 ? seed : seed / area;
  const int prec = x->L.prec, flow = x->L.flow;
  // the seed stores S^T lambda_T, with the dL/dT_w terms of the last step
  HIPCHK(x, prec == 0 ? launch_adj_seed<0>(cp, n, flow, scale, x->region[x->cur], lam[0], dtw, x->stream)
                      : launch_adj_seed<1>(cp, n, flow, scale, x->region[x->cur], lam[0], dtw, x->stream));
  int li = 0;  // lam[li] holds S^T lambda at the current time (lambda_0 itself at the end)
  auto state_at = [&](int64_t t, int64_t t0) -> char* {
    const int64_t seg = t0 / a.every;
    if (t == t0) return a.ws + a.o_snap + rb * static_cast<size_t>(seg);
    return a.ws + a.o_seg + rb * static_cast<size_t>(t - t0 - 1);
  };
  for (int seg = a.nsnap - 1; seg >= 0; --seg) {
    const int64_t t0 = static_cast<int64_t>(seg) * a.every;
    const int64_t t1 = std::min<int64_t>(t0 + a.every, a.nsteps);
    // recompute the states t0+1 .. t1-1 of this segment from its snapshot
    // (the forward run left those of the last segment in place)
    const bool kept = seg == a.nsnap - 1 && a.last_seg_kept;
    if (!kept && t1 - t0 > 1) a.last_seg_kept = false;  // the slots now hold another segment
    for (int64_t t = t0; !kept && t + 1 < t1; ++t)
      HIPCHK(x, dispatch_step(x, state_at(t, t0), state_at(t + 1, t0), nullptr, 0, x->stream));
    for (int64_t t = t1 - 1; t >= t0; --t) {
      AdjArgs g;
      g.cavs = x->d_params;
      g.tiles = x->d_tiles;
      g.ntiles = x->ntiles;
      g.state = state_at(t, t0);
      g.lam_in = lam[li];
      g.lam_out = lam[li ^ 1];
      g.dTw = dtw;
      g.block = x->block;
      g.reverse = li;  // alternates from one adjoint step to the next
      g.last = t == 0;
      g.flow = flow;
      g.mrt = x->L.mrt;
      g.stream = x->stream;
      HIPCHK(x, prec == 0 ? launch_adjoint<0>(g) : launch_adjoint<1>(g));
      li ^= 1;
    }
  }
  if (dev_dL_dTw)
    HIPCHK(x, hipMemcpyAsync(dev_dL_dTw, dtw, sizeof(double) * x->L.tw_doubles,
                             hipMemcpyDeviceToDevice, x->stream));
  if (dev_dL_dT0)
    HIPCHK(x, prec == 0 ? launch_adj_T0<0>(cp, n, flow, a.ws + a.o_snap, lam[li], dev_dL_dT0, x->stream)
                        : launch_adj_T0<1>(cp, n, flow, a.ws + a.o_snap, lam[li], dev_dL_dT0, x->stream));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  return LBPC_OK;
}

int lbpc_adjoint(lbpc_ctx* x, int64_t nsteps, int32_t every, int32_t loss, void* dev_adj_ws,
                 size_t bytes, double* dev_dL_dTw, double* dev_dL_dT0, double* host_loss) {
  const int rc = lbpc_adjoint_forward(x, nsteps, every, loss, dev_adj_ws, bytes, host_loss);
  if (rc) return rc;
  return lbpc_adjoint_backward(x, 1.0, dev_dL_dTw, dev_dL_dT0);
}

}  // extern "C"

// Device code of the coupled D3Q19 / D3Q7 phase-change lattice Boltzmann step
// (Li & He, arXiv 1703.02652) for gfx950.  Included by the per-format kernel
// translation units only.
//
// Layout: every cavity owns, inside a state region, 19 f planes, 6 planes for
// g_1..g_6 and one plane for g_0 (followed by its int16 correction plane in
// the FP32 format), each plane `plane` elements long, cell index
// x + nx (y + ny z).  FP64 stores the populations as they are; the other
// formats store f_a - w_a rho0 (deviation from rest), the 16-bit ones also
// g_a relative to a reference (kShiftG); g_0 is FP64, FP32 + correction
// (kSplitG0) or FP32 in the 16-bit formats.
//
// Step scheme: one thread per cell reads its own pre-collision populations
// (aligned, coalesced), does both collisions in registers and pushes every
// post-collision population to the cell it streams to (a bijection, so no
// write conflicts).  The stored state is therefore always the pre-collision
// state of Eq. (5) / Eq. (50), the one the fields and the adjoint are defined on.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbpc_api.hpp"

namespace lbpc {

// ---------------------------------------------------------------------------
// Storage formats
// ---------------------------------------------------------------------------
template <int P> struct Fmt;
// g_0 carries the latent heat (h = g_0 + sum of the small moving populations):
// FP32 alone would round the small per-step enthalpy changes of a mushy cell
// away against its large value over long runs.  The FP32 format therefore
// stores g_0 as an FP32 value and a 16-bit correction (kSplitG0, 6 bytes, 40
// significant bits; see g0_join), FP64 stores it as it is, and the 16-bit
// formats in FP32: their own rounding of the moving populations is far larger
// than what FP32 g_0 loses.
template <> struct Fmt<P64> { using S = double;   using S0 = double; using R = double; };
template <> struct Fmt<P32> { using S = float;    using S0 = float;  using R = float; };
template <> struct Fmt<P16> { using S = _Float16; using S0 = float;  using R = float; };
template <> struct Fmt<PB16> { using S = __bf16;  using S0 = float;  using R = float; };
template <int P> constexpr bool kSplitG0 = P == P32;

// g_0 of the FP32 format: hi = g_0 rounded to FP32, lo = the rest in units of
// ulp(hi) / 2^16, rounded to an int16 (|rest| <= ulp(hi) / 2, so |lo| <=
// 2^15).  g_0 = hi + lo * ulp(hi) / 2^16 to within ulp(hi) / 2^17, i.e. 40
// significant bits.  Zero and FP32 subnormals use the subnormal ulp.
__device__ __forceinline__ int g0_lo_exp(float hi) {
  const uint32_t e = (__float_as_uint(hi) >> 23) & 0xffu;
  return static_cast<int>(e == 0u ? 1u : e) - 127 - 23 - 16;
}
__device__ __forceinline__ double pow2(int k) {  // 2^k for -1022 <= k <= 1023
  return __longlong_as_double(static_cast<long long>(k + 1023) << 52);
}
__device__ __forceinline__ double g0_join(float hi, int16_t lo) {
  return static_cast<double>(hi) + static_cast<double>(lo) * pow2(g0_lo_exp(hi));
}
__device__ __forceinline__ void g0_split(double v, float& hi, int16_t& lo) {
  hi = static_cast<float>(v);
  // v - hi is exact in FP64; scaling by a power of two is exact
  const double q = rint((v - static_cast<double>(hi)) * pow2(-g0_lo_exp(hi)));
  lo = static_cast<int16_t>(fmin(fmax(q, -32768.0), 32767.0));
}

// The 16-bit formats store the moving enthalpy populations as deviations from
// a reference, g_a - (omega_T / 2) C_p,ref T_shift (a = 1..6), which spends
// their few mantissa bits on what differs from it; the other formats store
// g_a.  Kernels work on the stored values and add the reference where the
// full populations enter (their sum h, the SRT equilibrium, the
// anti-bounce-back rule).
template <int P> constexpr bool kShiftG = P == P16 || P == PB16;

__device__ __forceinline__ double dec(double v) { return v; }
__device__ __forceinline__ float dec(float v) { return v; }
__device__ __forceinline__ float dec(_Float16 v) { return static_cast<float>(v); }
__device__ __forceinline__ float dec(__bf16 v) { return static_cast<float>(v); }

template <class S> __device__ __forceinline__ S enc(double v);
template <> __device__ __forceinline__ double enc<double>(double v) { return v; }
template <> __device__ __forceinline__ float enc<float>(double v) { return static_cast<float>(v); }
template <> __device__ __forceinline__ _Float16 enc<_Float16>(double v) {
  return static_cast<_Float16>(static_cast<float>(v));
}
template <> __device__ __forceinline__ __bf16 enc<__bf16>(double v) {
  return static_cast<__bf16>(static_cast<float>(v));  // round to nearest even
}

// Streaming loads: each stored population is read exactly once per step, so
// the loads carry the non-temporal hint (they need not stay in the caches).
template <class S> __device__ __forceinline__ S ld_stream(const S* p) {
  return __builtin_nontemporal_load(p);
}
template <> __device__ __forceinline__ __bf16 ld_stream<__bf16>(const __bf16* p) {
  const uint16_t b = __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p));
  return __builtin_bit_cast(__bf16, b);
}

// Population planes through buffer resources (step kernel).  A plane is
// addressed by a resource holding its base and byte size (scalar registers)
// and one 32-bit byte offset per lane.  The hardware range check drops a store
// whose offset is at or past the plane size, so a lane is masked out of a
// store by giving it the offset kDrop.  Planes hold fewer than 2^29 cells of at
// most 8 bytes, so every plane size stays below kDrop.
constexpr uint32_t kDrop = 0xFFFFFFF0u;
constexpr int kNonTemporal = 2;   // cache-policy bits of a streaming load

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, uint32_t bytes) {
  // word 3: raw access (no swizzle, stride 0) with a 32-bit data format
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, static_cast<int>(bytes),
                                           0x00020000);
}
template <class S> __device__ __forceinline__ S buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <class S> __device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, S v);
template <> __device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                        r, static_cast<int>(off), 0, kNonTemporal));
}
template <> __device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                       r, static_cast<int>(off), 0, kNonTemporal));
}
template <> __device__ __forceinline__ _Float16 buf_ld<_Float16>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(
                                          r, static_cast<int>(off), 0, kNonTemporal));
}
template <> __device__ __forceinline__ __bf16 buf_ld<__bf16>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(
                                        r, static_cast<int>(off), 0, kNonTemporal));
}
template <> __device__ __forceinline__ int16_t buf_ld<int16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(int16_t, __builtin_amdgcn_raw_buffer_load_b16(
                                         r, static_cast<int>(off), 0, kNonTemporal));
}
template <> __device__ __forceinline__ void buf_st<int16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off, int16_t v) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, static_cast<int>(off), 0, 0);
}
template <> __device__ __forceinline__ void buf_st<double>(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  using B = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B, v), r, static_cast<int>(off), 0, 0);
}
template <> __device__ __forceinline__ void buf_st<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, static_cast<int>(off), 0, 0);
}
template <> __device__ __forceinline__ void buf_st<_Float16>(__amdgpu_buffer_rsrc_t r, uint32_t off, _Float16 v) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, static_cast<int>(off), 0, 0);
}
template <> __device__ __forceinline__ void buf_st<__bf16>(__amdgpu_buffer_rsrc_t r, uint32_t off, __bf16 v) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, static_cast<int>(off), 0, 0);
}

template <int P> struct View {
  using S = typename Fmt<P>::S;
  using S0 = typename Fmt<P>::S0;
  S* f;     // 19 planes (only with flow)
  S* g;     // g_1..g_6 planes
  S0* g0;   // g_0 plane (the FP32 part in the FP32 format)
  int16_t* g0lo;  // FP32 format: the correction plane of g_0 (kSplitG0)
  int64_t plane;
};

template <int P>
__device__ __forceinline__ View<P> view(const char* region, const CavParams& c, bool flow) {
  using S = typename Fmt<P>::S;
  using S0 = typename Fmt<P>::S0;
  View<P> v;
  v.plane = c.plane;
  v.f = reinterpret_cast<S*>(const_cast<char*>(region) + c.off);
  v.g = v.f + (flow ? 19 * c.plane : 0);
  v.g0 = reinterpret_cast<S0*>(v.g + 6 * c.plane);
  v.g0lo = reinterpret_cast<int16_t*>(v.g0 + c.plane);
  return v;
}

// g_0 of one cell as FP64, and its store, for the kernels that address the
// planes through plain pointers.
template <int P> __device__ __forceinline__ double load_g0(const View<P>& v, int32_t cell) {
  if constexpr (kSplitG0<P>) return g0_join(v.g0[cell], v.g0lo[cell]);
  else return static_cast<double>(v.g0[cell]);
}
template <int P> __device__ __forceinline__ void store_g0(const View<P>& v, int32_t cell, double x) {
  if constexpr (kSplitG0<P>) {
    float hi;
    int16_t lo;
    g0_split(x, hi, lo);
    v.g0[cell] = hi;
    v.g0lo[cell] = lo;
  } else {
    v.g0[cell] = static_cast<typename Fmt<P>::S0>(x);
  }
}

// ---------------------------------------------------------------------------
// Lattices (velocity order of Eq. (48) for D3Q19 and Eq. (3) for D3Q7)
// ---------------------------------------------------------------------------
constexpr int Q19X[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int Q19Y[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int Q19Z[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int Q19OPP[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
constexpr int Q7X[7] = {0, 1, -1, 0, 0, 0, 0};
constexpr int Q7Y[7] = {0, 0, 0, 1, -1, 0, 0};
constexpr int Q7Z[7] = {0, 0, 0, 0, 0, 1, -1};
constexpr int Q7OPP[7] = {0, 2, 1, 4, 3, 6, 5};
// D3Q19 rest weights (equilibrium at u = 0: 1/3, 1/18, 1/36)
constexpr double W19[19] = {1.0 / 3, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

__device__ __forceinline__ uint32_t fastdiv(uint32_t i, uint64_t m, uint32_t s) {
  return static_cast<uint32_t>((static_cast<uint64_t>(i) * m) >> s);
}

struct Site {
  int32_t x, y, z, cell;
  bool lx, hx, ly, hy, lz, hz;
};

__device__ __forceinline__ Site make_site(const CavParams& c, int32_t cell) {
  Site s;
  s.cell = cell;
  s.z = static_cast<int32_t>(fastdiv(static_cast<uint32_t>(cell), c.div_nxy_m, c.div_nxy_s));
  const int32_t r = cell - s.z * c.nxy;
  s.y = static_cast<int32_t>(fastdiv(static_cast<uint32_t>(r), c.div_nx_m, c.div_nx_s));
  s.x = r - s.y * c.nx;
  s.lx = s.x == 0;
  s.hx = s.x == c.nx - 1;
  s.ly = s.y == 0;
  s.hy = s.y == c.ny - 1;
  s.lz = s.z == 0;
  s.hz = s.z == c.nz - 1;
  return s;
}

// Cell reached by moving one link (ex, ey, ez) from s; periodic faces wrap.
// face >= 0 when the link leaves through a non-periodic face (the last such
// face for a diagonal that crosses two).
__device__ __forceinline__ int32_t link_target(const CavParams& c, const Site& s, int ex, int ey,
                                               int ez, int& face) {
  int32_t idx = s.cell + ex + ey * c.nx + ez * c.nxy;
  face = -1;
  if (ex > 0 && s.hx) { if (c.bc[1] == BC_PERIODIC) idx -= c.nx; else face = 1; }
  if (ex < 0 && s.lx) { if (c.bc[0] == BC_PERIODIC) idx += c.nx; else face = 0; }
  if (ey > 0 && s.hy) { if (c.bc[3] == BC_PERIODIC) idx -= c.nxy; else face = 3; }
  if (ey < 0 && s.ly) { if (c.bc[2] == BC_PERIODIC) idx += c.nxy; else face = 2; }
  if (ez > 0 && s.hz) { if (c.bc[5] == BC_PERIODIC) idx -= c.n; else face = 5; }
  if (ez < 0 && s.lz) { if (c.bc[4] == BC_PERIODIC) idx += c.n; else face = 4; }
  return idx;
}

// True when the link (ex, ey, ez) from s leaves the cavity (all faces walls).
__device__ __forceinline__ bool hits_wall(const Site& s, int ex, int ey, int ez) {
  return (ex > 0 && s.hx) || (ex < 0 && s.lx) || (ey > 0 && s.hy) || (ey < 0 && s.ly) ||
         (ez > 0 && s.hz) || (ez < 0 && s.lz);
}

// Node of a face field seen by the cell at s: x faces [nz][ny], y faces
// [nz][nx], z faces [ny][nx].
__device__ __forceinline__ int64_t face_node(const CavParams& c, const Site& s, int face) {
  const int dim = face >> 1;
  if (dim == 0) return s.y + static_cast<int64_t>(c.ny) * s.z;
  if (dim == 1) return s.x + static_cast<int64_t>(c.nx) * s.z;
  return s.x + static_cast<int64_t>(c.nx) * s.y;
}

// ---------------------------------------------------------------------------
// Cell physics
// ---------------------------------------------------------------------------
// Enthalpy -> (T, f_l), Eq. (2) with h0 = 0, as the lever rule: solid for
// h <= h_s = C_p,s T_m, liquid for h >= h_l = C_p,l T_m + L, isothermal at T_m
// in between.  FP64 for every storage format.
__device__ __forceinline__ void phase_rule(const CavParams& c, double h, double& T, double& fl) {
  if (h <= c.hs) {
    fl = 0.0;
    T = h * c.inv_cps;
  } else if (h >= c.hl) {
    fl = 1.0;
    T = (h - c.latent) * c.inv_cpl;
  } else {
    fl = (h - c.hs) * c.inv_dh;
    T = c.T_m;
  }
}

// Sum of the six moving enthalpy populations (compute type) and h = g_0 + that
// sum in FP64.  Every kernel that needs h of a cell goes through this, so the
// step, its adjoint and the diagnostics take the same phase branch.
template <class R> __device__ __forceinline__ R moving_sum(const R* g) {
  return ((g[1] + g[2]) + (g[3] + g[4])) + (g[5] + g[6]);
}

// Macroscopic flow variables and forces of one cell (Eq. (55), (56)) with the
// solid-region forcing u = f_l j / rho, j = sum f e + F_b / 2; d holds the
// stored deviations f - fshift w.
template <class R> struct FlowMacro {
  R dr, rho, jx, jy, jz0, ux, uy, uz, Fx, Fy, Fz;
};

template <class R>
__device__ __forceinline__ FlowMacro<R> flow_macro(const CavParams& c, const R* d, R T, R fl) {
  FlowMacro<R> m;
  R dr = d[0];
  R jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int a = 1; a < 19; ++a) {
    dr += d[a];
    if (Q19X[a] != 0) jx += Q19X[a] > 0 ? d[a] : -d[a];
    if (Q19Y[a] != 0) jy += Q19Y[a] > 0 ? d[a] : -d[a];
    if (Q19Z[a] != 0) jz += Q19Z[a] > 0 ? d[a] : -d[a];
  }
  m.dr = dr;
  const Pars<R>& k = pars<R>(c);
  m.rho = k.fshift + dr;
  m.jx = jx;
  m.jy = jy;
  m.jz0 = jz;
  const R Fb = k.g_beta_rho0 * (T - k.T_ref);
  const R jzb = jz + static_cast<R>(0.5) * Fb;
  const R irho = static_cast<R>(1) / m.rho;
  m.ux = fl * jx * irho;
  m.uy = fl * jy * irho;
  m.uz = fl * jzb * irho;
  m.Fx = static_cast<R>(2) * (m.rho * m.ux - jx);
  m.Fy = static_cast<R>(2) * (m.rho * m.uy - jy);
  m.Fz = static_cast<R>(2) * (m.rho * m.uz - jz);
  return m;
}

// D3Q19 MRT collision with forcing, Eq. (49)-(54), in registers.  The moment
// basis of Eq. (51) is applied as grouped sums (axis pairs and the three
// diagonal families); M^-1 = M^T diag(1/|row|^2) because the rows are
// orthogonal.  Working on deviations d = f - fshift w is exact algebra: the
// rest state contributes only to the rho, e and epsilon moments.
template <class R>
__device__ __forceinline__ void flow_collide(const CavParams& c, R* d, const FlowMacro<R>& q) {
  const R sx = d[1] + d[2], ax = d[1] - d[2];
  const R sy = d[3] + d[4], ay = d[3] - d[4];
  const R sz = d[5] + d[6], az = d[5] - d[6];
  const R p78 = d[7] + d[8], m78 = d[7] - d[8], p910 = d[9] + d[10], m910 = d[9] - d[10];
  const R Sxy = p78 + p910, Axy_x = m78 + m910, Axy_y = p78 - p910, Pxy = m78 - m910;
  const R p1112 = d[11] + d[12], m1112 = d[11] - d[12], p1314 = d[13] + d[14], m1314 = d[13] - d[14];
  const R Sxz = p1112 + p1314, Axz_x = m1112 + m1314, Axz_z = p1112 - p1314, Pxz = m1112 - m1314;
  const R p1516 = d[15] + d[16], m1516 = d[15] - d[16], p1718 = d[17] + d[18], m1718 = d[17] - d[18];
  const R Syz = p1516 + p1718, Ayz_y = m1516 + m1718, Ayz_z = p1516 - p1718, Pyz = m1516 - m1718;
  const R Sax = sx + sy + sz, Sdg = Sxy + Sxz + Syz;

  const R m1 = static_cast<R>(-30) * d[0] + static_cast<R>(-11) * Sax + static_cast<R>(8) * Sdg;
  const R m2 = static_cast<R>(12) * d[0] + static_cast<R>(-4) * Sax + Sdg;
  const R m4 = static_cast<R>(-4) * ax + Axy_x + Axz_x;
  const R m6 = static_cast<R>(-4) * ay + Axy_y + Ayz_y;
  const R m8 = static_cast<R>(-4) * az + Axz_z + Ayz_z;
  const R m9 = static_cast<R>(2) * sx - sy - sz + Sxy + Sxz - static_cast<R>(2) * Syz;
  const R m10 = static_cast<R>(-4) * sx + static_cast<R>(2) * (sy + sz) + Sxy + Sxz -
                static_cast<R>(2) * Syz;
  const R m11 = sy - sz + Sxy - Sxz;
  const R m12 = static_cast<R>(-2) * (sy - sz) + Sxy - Sxz;
  const R m16 = Axy_x - Axz_x, m17 = Ayz_y - Axy_y, m18 = Axz_z - Ayz_z;

  const R rho = q.rho, ux = q.ux, uy = q.uy, uz = q.uz, Fx = q.Fx, Fy = q.Fy, Fz = q.Fz;
  const R u2 = ux * ux + uy * uy + uz * uz;
  const R Fu = Fx * ux + Fy * uy + Fz * uz;
  const Pars<R>& pk = pars<R>(c);
  const R s_e = pk.s_e, s_eps = pk.s_eps, s_q = pk.s_q;
  const R s_nu = pk.s_nu, s_pi = pk.s_pi, s_t = pk.s_t;
  const R half = static_cast<R>(0.5), one = static_cast<R>(1);
  const R k_e = one - half * s_e, k_eps = one - half * s_eps, k_q = one - half * s_q;
  const R k_nu = one - half * s_nu, k_pi = one - half * s_pi;
  const R two3 = static_cast<R>(2.0 / 3.0);
  const R p9 = static_cast<R>(3) * ux * ux - u2;
  const R p11 = uy * uy - uz * uz;

  // Delta_k = Lambda_k (m_k - m_k^eq) - (1 - Lambda_k / 2) FF_k, scaled by 1/|row_k|^2
  const R a1 = (s_e * (m1 + static_cast<R>(11) * q.dr - static_cast<R>(19) * rho * u2) -
                k_e * static_cast<R>(38) * Fu) * static_cast<R>(1.0 / 2394.0);
  const R a2 = (s_eps * (m2 - static_cast<R>(3) * q.dr + static_cast<R>(5.5) * rho * u2) +
                k_eps * static_cast<R>(11) * Fu) * static_cast<R>(1.0 / 252.0);
  const R a3 = -Fx * static_cast<R>(0.1);
  const R a5 = -Fy * static_cast<R>(0.1);
  const R a7 = -Fz * static_cast<R>(0.1);
  const R a4 = (s_q * (m4 + two3 * rho * ux) + k_q * two3 * Fx) * static_cast<R>(1.0 / 40.0);
  const R a6 = (s_q * (m6 + two3 * rho * uy) + k_q * two3 * Fy) * static_cast<R>(1.0 / 40.0);
  const R a8 = (s_q * (m8 + two3 * rho * uz) + k_q * two3 * Fz) * static_cast<R>(1.0 / 40.0);
  const R a9 = (s_nu * (m9 - rho * p9) - k_nu * (static_cast<R>(6) * Fx * ux - static_cast<R>(2) * Fu)) *
               static_cast<R>(1.0 / 36.0);
  const R a10 = (s_pi * (m10 + half * rho * p9) - k_pi * (Fu - static_cast<R>(3) * Fx * ux)) *
                static_cast<R>(1.0 / 72.0);
  const R a11 = (s_nu * (m11 - rho * p11) - k_nu * static_cast<R>(2) * (Fy * uy - Fz * uz)) *
                static_cast<R>(1.0 / 12.0);
  const R a12 = (s_pi * (m12 + half * rho * p11) - k_pi * (Fz * uz - Fy * uy)) *
                static_cast<R>(1.0 / 24.0);
  const R a13 = (s_nu * (Pxy - rho * ux * uy) - k_nu * (Fx * uy + Fy * ux)) * static_cast<R>(0.25);
  const R a14 = (s_nu * (Pyz - rho * uy * uz) - k_nu * (Fy * uz + Fz * uy)) * static_cast<R>(0.25);
  const R a15 = (s_nu * (Pxz - rho * ux * uz) - k_nu * (Fx * uz + Fz * ux)) * static_cast<R>(0.25);
  const R a16 = s_t * m16 * static_cast<R>(0.125);
  const R a17 = s_t * m17 * static_cast<R>(0.125);
  const R a18 = s_t * m18 * static_cast<R>(0.125);

  // f* = f - M^T a
  d[0] -= static_cast<R>(-30) * a1 + static_cast<R>(12) * a2;
  const R A = static_cast<R>(-11) * a1 + static_cast<R>(-4) * a2;
  const R X1 = a3 - static_cast<R>(4) * a4, Y1 = a5 - static_cast<R>(4) * a6,
          Z1 = a7 - static_cast<R>(4) * a8;
  const R Pxx = static_cast<R>(2) * a9 - static_cast<R>(4) * a10;
  const R Pyy = -a9 + static_cast<R>(2) * a10 + a11 - static_cast<R>(2) * a12;
  const R Pzz = -a9 + static_cast<R>(2) * a10 - a11 + static_cast<R>(2) * a12;
  d[1] -= A + X1 + Pxx;
  d[2] -= A - X1 + Pxx;
  d[3] -= A + Y1 + Pyy;
  d[4] -= A - Y1 + Pyy;
  d[5] -= A + Z1 + Pzz;
  d[6] -= A - Z1 + Pzz;
  const R D = static_cast<R>(8) * a1 + a2;
  const R Dxy = D + a9 + a10 + a11 + a12, X2 = a3 + a4 + a16, Y2 = a5 + a6 - a17;
  d[7] -= Dxy + X2 + Y2 + a13;
  d[8] -= Dxy - X2 + Y2 - a13;
  d[9] -= Dxy + X2 - Y2 - a13;
  d[10] -= Dxy - X2 - Y2 + a13;
  const R Dxz = D + a9 + a10 - a11 - a12, X3 = a3 + a4 - a16, Z3 = a7 + a8 + a18;
  d[11] -= Dxz + X3 + Z3 + a15;
  d[12] -= Dxz - X3 + Z3 - a15;
  d[13] -= Dxz + X3 - Z3 - a15;
  d[14] -= Dxz - X3 - Z3 + a15;
  const R Dyz = D - static_cast<R>(2) * (a9 + a10), Y4 = a5 + a6 + a17, Z4 = a7 + a8 - a18;
  d[15] -= Dyz + Y4 + Z4 + a14;
  d[16] -= Dyz - Y4 + Z4 - a14;
  d[17] -= Dyz + Y4 - Z4 - a14;
  d[18] -= Dyz - Y4 - Z4 + a14;
}

// Thermal relaxation rate of a cell: sigma_chi = 1 / tau_g, tau_g = chi / omega_T
// + 1/2 with chi = lambda(f_l) / (rho0 C_p,ref) (Eq. (20), (34)).
template <class R>
__device__ __forceinline__ R sigma_chi(const CavParams& c, R fl) {
  const Pars<R>& k = pars<R>(c);
  const R lam = k.lam_s + fl * k.dlam;
  return static_cast<R>(1) / (lam * k.inv_rcw + static_cast<R>(0.5));
}

// MRT rates (Eq. (23), (47)): sigma_1..3 = sigma_chi, sigma_4..6 = 2 - sigma_chi,
// each replaceable by a fixed override.
template <class R>
__device__ __forceinline__ void mrt_rates(const CavParams& c, R sig, R* r) {
  r[1] = r[2] = r[3] = sig;
  r[4] = r[5] = r[6] = static_cast<R>(2) - sig;
  if (c.has_override) {
#pragma unroll
    for (int k = 1; k < 7; ++k)
      if (!isnan(c.sig_ovr[k])) r[k] = pars<R>(c).sig_ovr[k];
  }
}

// D3Q7 MRT collision, Eq. (21)-(25).  n_4 - n_4^eq is formed as
// -7 sum_{a>0} g_a + 21 omega_T C_p,ref T (the g_0 terms cancel exactly), which
// keeps the latent-heat-sized g_0 out of the difference.  g_1..g_6 are updated
// in place; the change of g_0 is returned (the caller adds it in FP64).
template <class R>
__device__ __forceinline__ R enth_collide_mrt(const CavParams& c, R* g, R s6, R T, R cp, R ux,
                                                 R uy, R uz, R sig) {
  R r[7];
  mrt_rates(c, sig, r);
  const R qT = cp * T;
  const R b1 = r[1] * (g[1] - g[2] - qT * ux) * static_cast<R>(0.5);
  const R b2 = r[2] * (g[3] - g[4] - qT * uy) * static_cast<R>(0.5);
  const R b3 = r[3] * (g[5] - g[6] - qT * uz) * static_cast<R>(0.5);
  const R b4 = r[4] * (static_cast<R>(-7) * s6 + pars<R>(c).w21 * T) *
               static_cast<R>(1.0 / 42.0);
  const R g12 = g[1] + g[2], g34 = g[3] + g[4], g56 = g[5] + g[6];
  const R b5 = r[5] * (static_cast<R>(2) * g12 - (g34 + g56)) * static_cast<R>(1.0 / 12.0);
  const R b6 = r[6] * (g34 - g56) * static_cast<R>(0.25);
  const R dg0 = -static_cast<R>(6) * b4;
  const R ax = -b4 + static_cast<R>(2) * b5;
  const R ay = -b4 - b5 + b6;
  const R az = -b4 - b5 - b6;
  g[1] -= ax + b1;
  g[2] -= ax - b1;
  g[3] -= ay + b2;
  g[4] -= ay - b2;
  g[5] -= az + b3;
  g[6] -= az - b3;
  return dg0;
}

// D3Q7 SRT (BGK) collision, Eq. (5)-(8): g^eq_0 = h - 3 omega_T C_p,ref T,
// g^eq_a = (omega_T / 2) C_p,ref T + (u.e_a / 2) C_p T.
template <class R, bool SHIFT = false>
__device__ __forceinline__ R enth_collide_srt(const CavParams& c, R* g, R s6, R T, R cp, R ux,
                                              R uy, R uz, R inv_tau) {
  R wT = pars<R>(c).whalf * T;
  if constexpr (SHIFT) wT -= pars<R>(c).gshift;  // g holds g_a - gshift
  const R hq = static_cast<R>(0.5) * cp * T;
  const R dg0 = -inv_tau * (pars<R>(c).w3 * T - s6);
  g[1] -= inv_tau * (g[1] - (wT + hq * ux));
  g[2] -= inv_tau * (g[2] - (wT - hq * ux));
  g[3] -= inv_tau * (g[3] - (wT + hq * uy));
  g[4] -= inv_tau * (g[4] - (wT - hq * uy));
  g[5] -= inv_tau * (g[5] - (wT + hq * uz));
  g[6] -= inv_tau * (g[6] - (wT - hq * uz));
  return dg0;
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Budget partials of one wavefront (global wave index = tile * waves per tile
// + wave, with the tile's place in the natural order of the cavities' cells,
// whatever the queue order), stored by its first lane; no workgroup barrier,
// so the waves of a tile retire without waiting for each other's population
// stores.
__device__ __forceinline__ int natural_tile(const CavParams& c, int2 tl) {
  return c.tile0 + tl.y / static_cast<int>(blockDim.x);
}
__device__ __forceinline__ int64_t wave_index(int tile) {
  return static_cast<int64_t>(tile) * (blockDim.x >> 6) + (threadIdx.x >> 6);
}
// wall inflow into the dense per-wavefront array of a ring slot
__device__ __forceinline__ void wave_inflow(double v, double* flux, int tile) {
  const double f = __any(v != 0.0) ? wave_sum(v) : 0.0;
  if ((threadIdx.x & 63) == 0) flux[wave_index(tile)] = f;
}
// the NPART sums of v into the wave's record (and the inflow sum into the
// slot's array when flux is given)
__device__ __forceinline__ void wave_sums(const double* v, double* sums, int tile,
                                          double* flux = nullptr) {
  double s[NPART];
#pragma unroll
  for (int k = 0; k < NPART; ++k) s[k] = wave_sum(v[k]);
  if ((threadIdx.x & 63) == 0) {
    const int64_t w = wave_index(tile);
    double* rec = sums + w * NPART;
#pragma unroll
    for (int k = 0; k < NPART; ++k) rec[k] = s[k];
    if (flux) flux[w] = s[3];
  }
}

// Queue position that workgroup slot t takes in a reversed walk: position
// t = kXcds j + k (XCD k) goes to the j-th last position of XCD k.
__device__ __forceinline__ int reversed_slot(int t, int ntiles) {
  const int k = t % kXcds, j = t / kXcds;
  const int per_xcd = (ntiles - k + kXcds - 1) / kXcds;  // positions of XCD k
  return (per_xcd - 1 - j) * kXcds + k;
}

// g_0 store through buffer resources (step kernel).
template <int P>
__device__ __forceinline__ void store_g0_buf(const View<P>& out, uint32_t pb0, uint32_t oc0,
                                             uint32_t pbl, uint32_t ocl, double x) {
  using S0 = typename Fmt<P>::S0;
  if constexpr (kSplitG0<P>) {
    float hi;
    int16_t lo;
    g0_split(x, hi, lo);
    buf_st<S0>(plane_rsrc(out.g0, pb0), oc0, hi);
    buf_st<int16_t>(plane_rsrc(out.g0lo, pbl), ocl, lo);
  } else {
    buf_st<S0>(plane_rsrc(out.g0, pb0), oc0, static_cast<S0>(x));
  }
}

// ---------------------------------------------------------------------------
// The fused step
// ---------------------------------------------------------------------------
// BUDGET: 0 no partials (recomputation inside the adjoint), 1 wall inflow only,
// 2 all partials (h, rho, f_l, wall inflow, bad cells).  reverse = 1 walks the
// queue positions of each XCD (those equal modulo kXcds) from their end:
// consecutive steps alternate, so that each XCD first reads what it wrote last
// in the step before, while that is still in its L2 and in the Infinity Cache,
// and every tile stays on one XCD from step to step.
template <int P, bool FLOW, bool MRT, int BUDGET>
__global__ void __launch_bounds__(256)
k_step(const CavParams* __restrict__ cavs, const int2* __restrict__ tiles, int ntiles, int reverse,
       const char* __restrict__ src, char* __restrict__ dst, double* __restrict__ partials,
       double* __restrict__ sums, const int32_t* __restrict__ status) {
  using S = typename Fmt<P>::S;
  using S0 = typename Fmt<P>::S0;
  using R = typename Fmt<P>::R;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int2 tl = tiles[reverse ? reversed_slot(t, ntiles) : t];
    const CavParams& c = cavs[tl.x];
    const int32_t cell = tl.y + static_cast<int32_t>(threadIdx.x);
    double acc[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (cell < c.n) {
      const View<P> in = view<P>(src, c, FLOW);
      const View<P> out = view<P>(dst, c, FLOW);
      const int64_t pl = c.plane;
      const uint32_t pb = static_cast<uint32_t>(pl) * static_cast<uint32_t>(sizeof(S));
      const uint32_t pb0 = static_cast<uint32_t>(pl) * static_cast<uint32_t>(sizeof(S0));
      const uint32_t oc = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S));
      const uint32_t oc0 = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S0));
      const uint32_t pbl = static_cast<uint32_t>(pl) * 2u, ocl = static_cast<uint32_t>(cell) * 2u;
      R d[19];
      R g[7];
      if (FLOW) {
#pragma unroll
        for (int a = 0; a < 19; ++a) d[a] = dec(buf_ld<S>(plane_rsrc(in.f + a * pl, pb), oc));
      }
      double g0d;
      if constexpr (kSplitG0<P>)
        g0d = g0_join(buf_ld<S0>(plane_rsrc(in.g0, pb0), oc0),
                      buf_ld<int16_t>(plane_rsrc(in.g0lo, pbl), ocl));
      else
        g0d = buf_ld<S0>(plane_rsrc(in.g0, pb0), oc0);
      g[0] = static_cast<R>(g0d);
#pragma unroll
      for (int a = 1; a < 7; ++a) g[a] = dec(buf_ld<S>(plane_rsrc(in.g + (a - 1) * pl, pb), oc));

      if (status[tl.x]) {  // frozen cavity: keep the state as it is
        if (FLOW) {
#pragma unroll
          for (int a = 0; a < 19; ++a) buf_st<S>(plane_rsrc(out.f + a * pl, pb), oc, enc<S>(d[a]));
        }
        store_g0_buf<P>(out, pb0, oc0, pbl, ocl, g0d);
#pragma unroll
        for (int a = 1; a < 7; ++a)
          buf_st<S>(plane_rsrc(out.g + (a - 1) * pl, pb), oc, enc<S>(g[a]));
      } else {
        // enthalpy -> (T, f_l) in FP64 (the moving populations are small; their
        // sum is formed in the compute type)
        R s6 = moving_sum(g);
        if constexpr (kShiftG<P>) s6 += static_cast<R>(6) * pars<R>(c).gshift;
        const double hd = g0d + static_cast<double>(s6);
        double Td, fld;
        phase_rule(c, hd, Td, fld);
        const R T = static_cast<R>(Td), fl = static_cast<R>(fld);
        const R cp = pars<R>(c).cp_s + fl * pars<R>(c).dcp;
        R ux = 0, uy = 0, uz = 0;
        double rhod = 0.0;
        bool bad = !isfinite(hd);
        if (FLOW) {
          const FlowMacro<R> q = flow_macro<R>(c, d, T, fl);
          ux = q.ux;
          uy = q.uy;
          uz = q.uz;
          rhod = static_cast<double>(c.fshift) + static_cast<double>(q.dr);
          bad = bad || !(rhod > 0.5 && rhod < 2.0) || !(ux * ux + uy * uy + uz * uz < R(0.09));
          flow_collide<R>(c, d, q);
        }
        const R sig = sigma_chi<R>(c, fl);
        const R dg0 = MRT ? enth_collide_mrt<R>(c, g, s6, T, cp, ux, uy, uz, sig)
                          : enth_collide_srt<R, kShiftG<P>>(c, g, s6, T, cp, ux, uy, uz, sig);

        // stream: push every post-collision population along its link.  With
        // walls on all six faces a link either stays inside the cavity (target
        // = this cell + a shift that is the same for the whole cavity) or hits
        // a wall; periodic faces go through link_target.
        const Site s = make_site(c, cell);
        if (FLOW) {
          buf_st<S>(plane_rsrc(out.f, pb), oc, enc<S>(d[0]));
          if (c.walls_only) {
#pragma unroll
            for (int a = 1; a < 19; ++a) {
              const S v = enc<S>(d[a]);
              const bool wall = hits_wall(s, Q19X[a], Q19Y[a], Q19Z[a]);
              const int32_t shift = Q19X[a] + Q19Y[a] * c.nx + Q19Z[a] * c.nxy;
              const uint32_t to = oc + static_cast<uint32_t>(shift) * static_cast<uint32_t>(sizeof(S));
              buf_st<S>(plane_rsrc(out.f + a * pl, pb), wall ? kDrop : to, v);
              if (wall) buf_st<S>(plane_rsrc(out.f + Q19OPP[a] * pl, pb), oc, v);  // halfway bounce-back
            }
          } else {
#pragma unroll
            for (int a = 1; a < 19; ++a) {
              int face;
              const int32_t to = link_target(c, s, Q19X[a], Q19Y[a], Q19Z[a], face);
              const S v = enc<S>(d[a]);
              if (face < 0)
                buf_st<S>(plane_rsrc(out.f + a * pl, pb),
                          static_cast<uint32_t>(to) * static_cast<uint32_t>(sizeof(S)), v);
              else
                buf_st<S>(plane_rsrc(out.f + Q19OPP[a] * pl, pb), oc, v);  // halfway bounce-back
            }
          }
        }
        store_g0_buf<P>(out, pb0, oc0, pbl, ocl, g0d + static_cast<double>(dg0));
        double flux = 0.0;
#pragma unroll
        for (int a = 1; a < 7; ++a) {
          const auto rs_out = plane_rsrc(out.g + (a - 1) * pl, pb);
          const auto rs_back = plane_rsrc(out.g + (Q7OPP[a] - 1) * pl, pb);
          int face;
          bool wall;
          if (c.walls_only) {
            face = (a & 1) ? a : a - 2;  // +x -> x+ face (1), -x -> x- face (0), ...
            wall = hits_wall(s, Q7X[a], Q7Y[a], Q7Z[a]);
            const int32_t shift = Q7X[a] + Q7Y[a] * c.nx + Q7Z[a] * c.nxy;
            const uint32_t to = oc + static_cast<uint32_t>(shift) * static_cast<uint32_t>(sizeof(S));
            buf_st<S>(rs_out, wall ? kDrop : to, enc<S>(g[a]));
          } else {
            const int32_t to = link_target(c, s, Q7X[a], Q7Y[a], Q7Z[a], face);
            wall = face >= 0;
            if (!wall)
              buf_st<S>(rs_out, static_cast<uint32_t>(to) * static_cast<uint32_t>(sizeof(S)),
                        enc<S>(g[a]));
          }
          if (wall) {
            if (c.bc[face] == BC_DIRICHLET) {
              // anti-bounce-back: g_abar(x) = -g*_a(x) + 2 w C_p,ref T_w
              const double Tw = c.tw[c.twface[face] + face_node(c, s, face)];
              R back = -g[a] + pars<R>(c).wabb * static_cast<R>(Tw);
              if constexpr (kShiftG<P>) back -= static_cast<R>(2) * pars<R>(c).gshift;
              buf_st<S>(rs_back, oc, enc<S>(back));
              flux += static_cast<double>(back) - static_cast<double>(g[a]);
            } else {
              buf_st<S>(rs_back, oc, enc<S>(g[a]));  // adiabatic
            }
          }
        }
        acc[0] = hd;
        acc[1] = rhod;
        acc[2] = fld;
        acc[3] = flux;
        acc[4] = bad ? 1.0 : 0.0;
      }
    }
    if (BUDGET == 1) wave_inflow(acc[3], partials, natural_tile(c, tl));
    if (BUDGET == 2) wave_sums(acc, sums, natural_tile(c, tl), partials);
  }
}

// Initial state at rest: f = w rho0 (stored deviation 0 in shifted formats),
// g = g^eq(h0(T0), T0, u = 0) with h0 from Eq. (2).
template <int P, bool FLOW>
__global__ void __launch_bounds__(256)
k_init(const CavParams* __restrict__ cavs, const int2* __restrict__ tiles, int ntiles,
       char* __restrict__ dst, const double* __restrict__ T0) {
  using S = typename Fmt<P>::S;
  using S0 = typename Fmt<P>::S0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int2 tl = tiles[t];
    const CavParams& c = cavs[tl.x];
    const int32_t cell = tl.y + static_cast<int32_t>(threadIdx.x);
    if (cell >= c.n) continue;
    const View<P> out = view<P>(dst, c, FLOW);
    const int64_t pl = c.plane;
    if (FLOW) {
#pragma unroll
      for (int a = 0; a < 19; ++a)
        out.f[a * pl + cell] = enc<S>(W19[a] * (c.rho0 - c.fshift));
    }
    const double T = T0 ? T0[c.cell_off + cell] : c.T_m;
    const double h0 = T <= c.T_m ? c.cp_s * T : c.cp_l * T + c.latent;
    store_g0<P>(out, cell, h0 - 3.0 * c.omega_T * c.cp_ref * T);
    double ga = 0.5 * c.omega_T * c.cp_ref * T;
    if constexpr (kShiftG<P>) ga -= c.gshift;
#pragma unroll
    for (int a = 1; a < 7; ++a) out.g[(a - 1) * pl + cell] = enc<S>(ga);
  }
}

// Sums of the current state per tile: h, rho, f_l, the enthalpy that the next
// step lets in through the x- face when it is a fixed-temperature face (the
// hot wall of the cavity workloads; each x = 0 cell recomputes its collision to
// get the outgoing g*_2 and applies the anti-bounce-back rule), bad cells.
template <int P, bool FLOW, bool MRT>
__global__ void __launch_bounds__(256)
k_measure(const CavParams* __restrict__ cavs, const int2* __restrict__ tiles, int ntiles,
          const char* __restrict__ src, double* __restrict__ partials) {
  using R = typename Fmt<P>::R;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int2 tl = tiles[t];
    const CavParams& c = cavs[tl.x];
    const int32_t cell = tl.y + static_cast<int32_t>(threadIdx.x);
    double acc[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (cell < c.n) {
      const View<P> in = view<P>(src, c, FLOW);
      const int64_t pl = c.plane;
      R d[19], g[7];
      if (FLOW) {
#pragma unroll
        for (int a = 0; a < 19; ++a) d[a] = dec(in.f[a * pl + cell]);
      }
      const double g0d = load_g0<P>(in, cell);
      g[0] = static_cast<R>(g0d);
#pragma unroll
      for (int a = 1; a < 7; ++a) g[a] = dec(in.g[(a - 1) * pl + cell]);
      R s6 = moving_sum(g);
      if constexpr (kShiftG<P>) s6 += static_cast<R>(6) * pars<R>(c).gshift;
      const double h = g0d + static_cast<double>(s6);
      double T, fl;
      phase_rule(c, h, T, fl);
      double rho = 0.0;
      FlowMacro<R> q;
      if (FLOW) {
        double dr = 0.0;
#pragma unroll
        for (int a = 0; a < 19; ++a) dr += static_cast<double>(d[a]);
        rho = c.fshift + dr;
        q = flow_macro<R>(c, d, static_cast<R>(T), static_cast<R>(fl));
      }
      const Site st = make_site(c, cell);
      if (st.lx && c.bc[0] == BC_DIRICHLET) {
        const R Tr = static_cast<R>(T), flr = static_cast<R>(fl);
        const R cp = static_cast<R>(c.cp_s) + flr * static_cast<R>(c.cp_l - c.cp_s);
        const R sig = sigma_chi<R>(c, flr);
        const R ux = FLOW ? q.ux : R(0), uy = FLOW ? q.uy : R(0), uz = FLOW ? q.uz : R(0);
        if (MRT) enth_collide_mrt<R>(c, g, s6, Tr, cp, ux, uy, uz, sig);
        else enth_collide_srt<R, kShiftG<P>>(c, g, s6, Tr, cp, ux, uy, uz, sig);
        const double Tw = c.tw[c.twface[0] + face_node(c, st, 0)];
        double g2 = static_cast<double>(g[2]);
        if constexpr (kShiftG<P>) g2 += c.gshift;
        acc[3] = c.omega_T * c.cp_ref * Tw - 2.0 * g2;
      }
      acc[0] = h;
      acc[1] = rho;
      acc[2] = fl;
      acc[4] = isfinite(h) && isfinite(rho) ? 0.0 : 1.0;
    }
    wave_sums(acc, partials, natural_tile(c, tl));
  }
}

// Fields of one cavity (FP64 planes in mask-bit order: h, T, f_l, rho, u).
template <int P, bool FLOW>
__global__ void __launch_bounds__(256)
k_fields(const CavParams* __restrict__ cavp, const char* __restrict__ src, uint32_t mask,
         double* __restrict__ out) {
  using R = typename Fmt<P>::R;
  const CavParams& c = *cavp;
  const int32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= c.n) return;
  const View<P> in = view<P>(src, c, FLOW);
  const int64_t pl = c.plane;
  R g[7];
#pragma unroll
  for (int a = 1; a < 7; ++a) g[a] = dec(in.g[(a - 1) * pl + cell]);
  R s6 = moving_sum(g);
  if constexpr (kShiftG<P>) s6 += static_cast<R>(6) * pars<R>(c).gshift;
  const double h = load_g0<P>(in, cell) + static_cast<double>(s6);
  double T, fl;
  phase_rule(c, h, T, fl);
  double rho = 0.0, u[3] = {0.0, 0.0, 0.0};
  if (FLOW) {
    R d[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) d[a] = dec(in.f[a * pl + cell]);
    const FlowMacro<R> q = flow_macro<R>(c, d, static_cast<R>(T), static_cast<R>(fl));
    rho = static_cast<double>(c.fshift) + static_cast<double>(q.dr);
    u[0] = q.ux;
    u[1] = q.uy;
    u[2] = q.uz;
  }
  int64_t k = 0;
  const int64_t n = c.n;
  if (mask & 1u) out[(k++) * n + cell] = h;
  if (mask & 2u) out[(k++) * n + cell] = T;
  if (mask & 4u) out[(k++) * n + cell] = fl;
  if (mask & 8u) out[(k++) * n + cell] = rho;
  if (mask & 16u) {
    out[(k++) * n + cell] = u[0];
    out[(k++) * n + cell] = u[1];
    out[(k++) * n + cell] = u[2];
  }
}

template <int P, bool FLOW>
__global__ void __launch_bounds__(256)
k_get_state(const CavParams* __restrict__ cavp, const char* __restrict__ src,
            double* __restrict__ f, double* __restrict__ g) {
  const CavParams& c = *cavp;
  const int32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= c.n) return;
  const View<P> in = view<P>(src, c, FLOW);
  const int64_t pl = c.plane, n = c.n;
  if (FLOW && f) {
#pragma unroll
    for (int a = 0; a < 19; ++a)
      f[a * n + cell] = static_cast<double>(dec(in.f[a * pl + cell])) + W19[a] * c.fshift;
  }
  g[cell] = load_g0<P>(in, cell);
#pragma unroll
  for (int a = 1; a < 7; ++a) {
    double v = static_cast<double>(dec(in.g[(a - 1) * pl + cell]));
    if constexpr (kShiftG<P>) v += c.gshift;
    g[a * n + cell] = v;
  }
}

template <int P, bool FLOW>
__global__ void __launch_bounds__(256)
k_set_state(const CavParams* __restrict__ cavp, char* __restrict__ dst,
            const double* __restrict__ f, const double* __restrict__ g) {
  using S = typename Fmt<P>::S;
  using S0 = typename Fmt<P>::S0;
  const CavParams& c = *cavp;
  const int32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= c.n) return;
  const View<P> out = view<P>(dst, c, FLOW);
  const int64_t pl = c.plane, n = c.n;
  if (FLOW) {
#pragma unroll
    for (int a = 0; a < 19; ++a) out.f[a * pl + cell] = enc<S>(f[a * n + cell] - W19[a] * c.fshift);
  }
  store_g0<P>(out, cell, g[cell]);
#pragma unroll
  for (int a = 1; a < 7; ++a) {
    double v = g[a * n + cell];
    if constexpr (kShiftG<P>) v -= c.gshift;
    out.g[(a - 1) * pl + cell] = enc<S>(v);
  }
}

}  // namespace lbpc

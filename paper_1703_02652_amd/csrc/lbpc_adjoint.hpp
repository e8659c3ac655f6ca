// Discrete adjoint of the fused step (device code).
//
// The step maps the pre-collision state s_t to s_{t+1} = S(C(s_t), T_w):
// a per-cell collision C followed by streaming S, which is a permutation of
// the post-collision populations except on fixed-temperature links, where
// g_abar(x) = -g*_a(x) + omega_T C_p,ref T_w.  For a loss of s_T the adjoint
// runs backwards, lambda_t = dC^T (S^T lambda_{t+1}):
//   - S^T: the adjoint of the post-collision population a at x is
//     lambda_a(x + e_a) for an interior link, lambda_abar(x) for a bounce-back
//     link and -lambda_abar(x) for an anti-bounce-back link, which also adds
//     omega_T C_p,ref lambda_abar(x) to dL/dT_w at that wall node.  It is
//     applied as a push when lambda is written: each adjoint step stores
//     M = S^T lambda_t (the transpose of the forward push is a pull, and a
//     pull of lambda_{t+1} is a push of lambda_t), so the next adjoint step
//     reads M aligned, as the forward step reads its state;
//   - dC^T is the transposed Jacobian of one cell update, written out by hand
//     below (reverse order of the forward cell update: enthalpy collision,
//     flow collision, forces and velocity, phase rule).  The phase rule is
//     piecewise linear in h; the branch of the forward pass is used, so the
//     kinks at h_s and h_l take the derivative of the closed side.
#pragma once
#include "lbpc_device.hpp"

namespace lbpc {

// Adjoint populations: planes of the compute type, 19 f planes (with flow)
// then g_0..g_6, at the same plane stride as the state.
template <class R> struct AdjView {
  R* f;
  R* g;
};
template <class R>
__device__ __forceinline__ AdjView<R> adj_view(const char* base, int64_t plane, bool flow) {
  AdjView<R> v;
  v.f = reinterpret_cast<R*>(const_cast<char*>(base));
  v.g = v.f + (flow ? 19 * plane : 0);
  return v;
}

// Store lambda_t(x) (lf: 19 flow, lg: 7 enthalpy components) as M = S^T
// lambda_t, which the adjoint step before it reads aligned: M_a(x - e_a) =
// lambda_a(x) for an interior link.  Where x - e_a lies outside, the link from
// x along e_abar hits a wall and lambda_a(x) goes to M_abar(x): as it is at a
// bounce-back or adiabatic link, negated at an anti-bounce-back link, which
// also adds omega_T C_p,ref lambda_a(x) to dL/dT_w of that wall node (one
// D3Q7 link crosses a face at each wall node, so one thread updates each
// accumulator per launch; single-cavity contexts, face fields from offset 0).
// Every slot of M is written exactly once.  natural: store lambda_t itself
// (the last adjoint step, whose result feeds dL/dT0).
template <class R, bool FLOW>
__device__ __forceinline__ void store_adjoint(const CavParams& c, const Site& s, const AdjView<R>& mo,
                                              int64_t pl, uint32_t pbr, uint32_t ocr, const R* lf,
                                              const R* lg, double* dTw, bool natural) {
  const uint32_t esz = static_cast<uint32_t>(sizeof(R));
  if (natural) {
    if (FLOW) {
#pragma unroll
      for (int a = 0; a < 19; ++a) buf_st<R>(plane_rsrc(mo.f + a * pl, pbr), ocr, lf[a]);
    }
#pragma unroll
    for (int a = 0; a < 7; ++a) buf_st<R>(plane_rsrc(mo.g + a * pl, pbr), ocr, lg[a]);
    return;
  }
  if (FLOW) {
    buf_st<R>(plane_rsrc(mo.f, pbr), ocr, lf[0]);
#pragma unroll
    for (int a = 1; a < 19; ++a) {
      bool wall;
      uint32_t to;
      if (c.walls_only) {
        wall = hits_wall(s, -Q19X[a], -Q19Y[a], -Q19Z[a]);
        const int32_t shift = Q19X[a] + Q19Y[a] * c.nx + Q19Z[a] * c.nxy;
        to = ocr - static_cast<uint32_t>(shift) * esz;
      } else {
        int face;
        const int32_t t = link_target(c, s, -Q19X[a], -Q19Y[a], -Q19Z[a], face);
        wall = face >= 0;
        to = static_cast<uint32_t>(t) * esz;
      }
      buf_st<R>(plane_rsrc(mo.f + a * pl, pbr), wall ? kDrop : to, lf[a]);
      if (wall) buf_st<R>(plane_rsrc(mo.f + Q19OPP[a] * pl, pbr), ocr, lf[a]);  // bounce-back
    }
  }
  buf_st<R>(plane_rsrc(mo.g, pbr), ocr, lg[0]);
#pragma unroll
  for (int a = 1; a < 7; ++a) {
    const int b = Q7OPP[a];
    int face;
    bool wall;
    uint32_t to;
    if (c.walls_only) {
      face = (b & 1) ? b : b - 2;  // face crossed along e_b: +x -> x+ (1), -x -> x- (0), ...
      wall = hits_wall(s, -Q7X[a], -Q7Y[a], -Q7Z[a]);
      const int32_t shift = Q7X[a] + Q7Y[a] * c.nx + Q7Z[a] * c.nxy;
      to = ocr - static_cast<uint32_t>(shift) * esz;
    } else {
      const int32_t t = link_target(c, s, -Q7X[a], -Q7Y[a], -Q7Z[a], face);
      wall = face >= 0;
      to = static_cast<uint32_t>(t) * esz;
    }
    buf_st<R>(plane_rsrc(mo.g + a * pl, pbr), wall ? kDrop : to, lg[a]);
    if (wall) {
      if (c.bc[face] == BC_DIRICHLET) {
        buf_st<R>(plane_rsrc(mo.g + b * pl, pbr), ocr, -lg[a]);
        const int64_t node = c.twface[face] + face_node(c, s, face);
        dTw[node] += c.omega_T * c.cp_ref * static_cast<double>(lg[a]);
      } else {
        buf_st<R>(plane_rsrc(mo.g + b * pl, pbr), ocr, lg[a]);
      }
    }
  }
}

// Transposed flow collision: given lf (adjoint of f*), accumulate into lf
// (becomes the adjoint of f through the moment path) and into the adjoints of
// rho, u and F.  Uses lf as an in/out array.
template <class R>
__device__ __forceinline__ void flow_collide_vjp(const CavParams& c, R* lf, const FlowMacro<R>& q,
                                                 R& rb, R& uxb, R& uyb, R& uzb, R& Fxb, R& Fyb,
                                                 R& Fzb, R& drb) {
  // mu = M lf (same grouped sums as the forward moments)
  const R* d = lf;
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
  const R mu1 = static_cast<R>(-30) * d[0] + static_cast<R>(-11) * Sax + static_cast<R>(8) * Sdg;
  const R mu2 = static_cast<R>(12) * d[0] + static_cast<R>(-4) * Sax + Sdg;
  const R mu3 = ax + Axy_x + Axz_x, mu5 = ay + Axy_y + Ayz_y, mu7 = az + Axz_z + Ayz_z;
  const R mu4 = static_cast<R>(-4) * ax + Axy_x + Axz_x;
  const R mu6 = static_cast<R>(-4) * ay + Axy_y + Ayz_y;
  const R mu8 = static_cast<R>(-4) * az + Axz_z + Ayz_z;
  const R mu9 = static_cast<R>(2) * sx - sy - sz + Sxy + Sxz - static_cast<R>(2) * Syz;
  const R mu10 = static_cast<R>(-4) * sx + static_cast<R>(2) * (sy + sz) + Sxy + Sxz -
                 static_cast<R>(2) * Syz;
  const R mu11 = sy - sz + Sxy - Sxz;
  const R mu12 = static_cast<R>(-2) * (sy - sz) + Sxy - Sxz;
  const R mu16 = Axy_x - Axz_x, mu17 = Ayz_y - Axy_y, mu18 = Axz_z - Ayz_z;

  // adjoint of Delta_k: f* = f - M^T diag(1/|row|^2) Delta  =>  Db_k = -mu_k / |row_k|^2
  const R D1 = -mu1 * static_cast<R>(1.0 / 2394.0), D2 = -mu2 * static_cast<R>(1.0 / 252.0);
  const R D3 = -mu3 * static_cast<R>(0.1), D5 = -mu5 * static_cast<R>(0.1), D7 = -mu7 * static_cast<R>(0.1);
  const R D4 = -mu4 * static_cast<R>(1.0 / 40.0), D6 = -mu6 * static_cast<R>(1.0 / 40.0),
          D8 = -mu8 * static_cast<R>(1.0 / 40.0);
  const R D9 = -mu9 * static_cast<R>(1.0 / 36.0), D10 = -mu10 * static_cast<R>(1.0 / 72.0);
  const R D11 = -mu11 * static_cast<R>(1.0 / 12.0), D12 = -mu12 * static_cast<R>(1.0 / 24.0);
  const R D13 = -Pxy * static_cast<R>(0.25), D14 = -Pyz * static_cast<R>(0.25),
          D15 = -Pxz * static_cast<R>(0.25);
  const R D16 = -mu16 * static_cast<R>(0.125), D17 = -mu17 * static_cast<R>(0.125),
          D18 = -mu18 * static_cast<R>(0.125);

  const R rho = q.rho, ux = q.ux, uy = q.uy, uz = q.uz, Fx = q.Fx, Fy = q.Fy, Fz = q.Fz;
  const R u2 = ux * ux + uy * uy + uz * uz;
  const R s_e = static_cast<R>(c.s_e), s_eps = static_cast<R>(c.s_eps), s_q = static_cast<R>(c.s_q);
  const R s_nu = static_cast<R>(c.s_nu), s_pi = static_cast<R>(c.s_pi), s_t = static_cast<R>(c.s_t);
  const R half = static_cast<R>(0.5), one = static_cast<R>(1);
  const R k_e = one - half * s_e, k_eps = one - half * s_eps, k_q = one - half * s_q;
  const R k_nu = one - half * s_nu, k_pi = one - half * s_pi;
  const R two3 = static_cast<R>(2.0 / 3.0);
  const R p9 = static_cast<R>(3) * ux * ux - u2;
  const R p11 = uy * uy - uz * uz;

  // direct moment path: lf += M^T psi with psi_k = Lambda_k Db_k
  const R q1 = s_e * D1, q2 = s_eps * D2, q4 = s_q * D4, q6 = s_q * D6, q8 = s_q * D8;
  const R q9 = s_nu * D9, q10 = s_pi * D10, q11 = s_nu * D11, q12 = s_pi * D12;
  const R q13 = s_nu * D13, q14 = s_nu * D14, q15 = s_nu * D15;
  const R q16 = s_t * D16, q17 = s_t * D17, q18 = s_t * D18;
  {
    R* o = lf;
    o[0] += static_cast<R>(-30) * q1 + static_cast<R>(12) * q2;
    const R A = static_cast<R>(-11) * q1 + static_cast<R>(-4) * q2;
    const R X1 = static_cast<R>(-4) * q4, Y1 = static_cast<R>(-4) * q6, Z1 = static_cast<R>(-4) * q8;
    const R Pxx = static_cast<R>(2) * q9 - static_cast<R>(4) * q10;
    const R Pyy = -q9 + static_cast<R>(2) * q10 + q11 - static_cast<R>(2) * q12;
    const R Pzz = -q9 + static_cast<R>(2) * q10 - q11 + static_cast<R>(2) * q12;
    o[1] += A + X1 + Pxx;
    o[2] += A - X1 + Pxx;
    o[3] += A + Y1 + Pyy;
    o[4] += A - Y1 + Pyy;
    o[5] += A + Z1 + Pzz;
    o[6] += A - Z1 + Pzz;
    const R Dg = static_cast<R>(8) * q1 + q2;
    const R Dxy = Dg + q9 + q10 + q11 + q12, X2 = q4 + q16, Y2 = q6 - q17;
    o[7] += Dxy + X2 + Y2 + q13;
    o[8] += Dxy - X2 + Y2 - q13;
    o[9] += Dxy + X2 - Y2 - q13;
    o[10] += Dxy - X2 - Y2 + q13;
    const R Dxz = Dg + q9 + q10 - q11 - q12, X3 = q4 - q16, Z3 = q8 + q18;
    o[11] += Dxz + X3 + Z3 + q15;
    o[12] += Dxz - X3 + Z3 - q15;
    o[13] += Dxz + X3 - Z3 - q15;
    o[14] += Dxz - X3 - Z3 + q15;
    const R Dyz = Dg - static_cast<R>(2) * (q9 + q10), Y4 = q6 + q17, Z4 = q8 - q18;
    o[15] += Dyz + Y4 + Z4 + q14;
    o[16] += Dyz - Y4 + Z4 - q14;
    o[17] += Dyz + Y4 - Z4 - q14;
    o[18] += Dyz - Y4 - Z4 + q14;
  }

  // equilibrium and forcing paths
  R u2b = 0, Fub = 0, p9b = 0, p11b = 0;
  drb += q1 * static_cast<R>(11) - q2 * static_cast<R>(3);
  rb += -q1 * static_cast<R>(19) * u2 + q2 * static_cast<R>(5.5) * u2;
  u2b += -q1 * static_cast<R>(19) * rho + q2 * static_cast<R>(5.5) * rho;
  Fub += -D1 * k_e * static_cast<R>(38) + D2 * k_eps * static_cast<R>(11);
  rb += two3 * (q4 * ux + q6 * uy + q8 * uz);
  uxb += two3 * q4 * rho;
  uyb += two3 * q6 * rho;
  uzb += two3 * q8 * rho;
  Fxb += two3 * k_q * D4;
  Fyb += two3 * k_q * D6;
  Fzb += two3 * k_q * D8;
  // Delta_9, Delta_10
  rb += -q9 * p9 + half * q10 * p9;
  p9b += -q9 * rho + half * q10 * rho;
  Fxb += -D9 * k_nu * static_cast<R>(6) * ux + D10 * k_pi * static_cast<R>(3) * ux;
  uxb += -D9 * k_nu * static_cast<R>(6) * Fx + D10 * k_pi * static_cast<R>(3) * Fx;
  Fub += D9 * k_nu * static_cast<R>(2) - D10 * k_pi;
  // Delta_11, Delta_12
  rb += -q11 * p11 + half * q12 * p11;
  p11b += -q11 * rho + half * q12 * rho;
  Fyb += -D11 * k_nu * static_cast<R>(2) * uy + D12 * k_pi * uy;
  uyb += -D11 * k_nu * static_cast<R>(2) * Fy + D12 * k_pi * Fy;
  Fzb += D11 * k_nu * static_cast<R>(2) * uz - D12 * k_pi * uz;
  uzb += D11 * k_nu * static_cast<R>(2) * Fz - D12 * k_pi * Fz;
  // Delta_13..15
  rb += -(q13 * ux * uy + q14 * uy * uz + q15 * ux * uz);
  uxb += -(q13 * rho * uy + D13 * k_nu * Fy) - (q15 * rho * uz + D15 * k_nu * Fz);
  uyb += -(q13 * rho * ux + D13 * k_nu * Fx) - (q14 * rho * uz + D14 * k_nu * Fz);
  uzb += -(q14 * rho * uy + D14 * k_nu * Fy) - (q15 * rho * ux + D15 * k_nu * Fx);
  Fxb += -D13 * k_nu * uy - D15 * k_nu * uz;
  Fyb += -D13 * k_nu * ux - D14 * k_nu * uz;
  Fzb += -D14 * k_nu * uy - D15 * k_nu * ux;
  // conserved moments: Delta_3,5,7 = -F
  Fxb += -D3;
  Fyb += -D5;
  Fzb += -D7;
  // p9 = 3 ux^2 - u2, p11 = uy^2 - uz^2, u2, F.u
  uxb += p9b * static_cast<R>(6) * ux;
  u2b += -p9b;
  uyb += p11b * static_cast<R>(2) * uy;
  uzb += -p11b * static_cast<R>(2) * uz;
  uxb += static_cast<R>(2) * ux * u2b + Fub * Fx;
  uyb += static_cast<R>(2) * uy * u2b + Fub * Fy;
  uzb += static_cast<R>(2) * uz * u2b + Fub * Fz;
  Fxb += Fub * ux;
  Fyb += Fub * uy;
  Fzb += Fub * uz;
}

template <int P, bool FLOW, bool MRT>
__global__ void __launch_bounds__(256)
k_adjoint(const CavParams* __restrict__ cavs, const int2* __restrict__ tiles, int ntiles, int reverse,
          int last, const char* __restrict__ state, const char* __restrict__ lam_in,
          char* __restrict__ lam_out, double* __restrict__ dTw) {
  using R = typename Fmt<P>::R;
  // consecutive adjoint steps walk the queue in opposite directions, as the
  // forward steps do: each XCD first reads the adjoint it wrote last
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int2 tl = tiles[reverse ? reversed_slot(t, ntiles) : t];
    const CavParams& c = cavs[tl.x];
    const int32_t cell = tl.y + static_cast<int32_t>(threadIdx.x);
    if (cell >= c.n) continue;
    const int64_t pl = c.plane;
    const View<P> st = view<P>(state, c, FLOW);
    const AdjView<R> li = adj_view<R>(lam_in, pl, FLOW);
    const AdjView<R> lo = adj_view<R>(lam_out, pl, FLOW);
    using S = typename Fmt<P>::S;
    using S0 = typename Fmt<P>::S0;
    // planes through buffer resources, as in the step kernel (32-bit offsets)
    const uint32_t pb = static_cast<uint32_t>(pl) * static_cast<uint32_t>(sizeof(S));
    const uint32_t pb0 = static_cast<uint32_t>(pl) * static_cast<uint32_t>(sizeof(S0));
    const uint32_t pbr = static_cast<uint32_t>(pl) * static_cast<uint32_t>(sizeof(R));
    const uint32_t oc = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S));
    const uint32_t oc0 = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S0));
    const uint32_t ocr = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(R));
    // ---- recompute the forward cell quantities
    R d[19], g[7];
    if (FLOW) {
#pragma unroll
      for (int a = 0; a < 19; ++a) d[a] = dec(buf_ld<S>(plane_rsrc(st.f + a * pl, pb), oc));
    }
    double g0d;
    if constexpr (kSplitG0<P>)
      g0d = g0_join(buf_ld<S0>(plane_rsrc(st.g0, pb0), oc0),
                    buf_ld<int16_t>(plane_rsrc(st.g0lo, static_cast<uint32_t>(pl) * 2u),
                                    static_cast<uint32_t>(cell) * 2u));
    else
      g0d = buf_ld<S0>(plane_rsrc(st.g0, pb0), oc0);
    g[0] = static_cast<R>(g0d);
#pragma unroll
    for (int a = 1; a < 7; ++a) g[a] = dec(buf_ld<S>(plane_rsrc(st.g + (a - 1) * pl, pb), oc));
    R s6 = moving_sum(g);
    if constexpr (kShiftG<P>) s6 += static_cast<R>(6) * pars<R>(c).gshift;
    const double hd = g0d + static_cast<double>(s6);
    double Td, fld;
    phase_rule(c, hd, Td, fld);
    // slopes of the phase rule on the branch taken
    R dT_dh, dfl_dh;
    if (hd <= c.hs) { dT_dh = static_cast<R>(c.inv_cps); dfl_dh = 0; }
    else if (hd >= c.hl) { dT_dh = static_cast<R>(c.inv_cpl); dfl_dh = 0; }
    else { dT_dh = 0; dfl_dh = static_cast<R>(c.inv_dh); }
    const R T = static_cast<R>(Td), fl = static_cast<R>(fld);
    const R cp = static_cast<R>(c.cp_s) + fl * static_cast<R>(c.cp_l - c.cp_s);
    FlowMacro<R> q;
    if (FLOW) q = flow_macro<R>(c, d, T, fl);
    const R ux = FLOW ? q.ux : R(0), uy = FLOW ? q.uy : R(0), uz = FLOW ? q.uz : R(0);
    const R sig = sigma_chi<R>(c, fl);

    // ---- the adjoint of the post-collision populations, M = S^T lambda_{t+1},
    // stored by the adjoint step after this one: aligned loads
    R lf[19], lg[7];
    if (FLOW) {
#pragma unroll
      for (int a = 0; a < 19; ++a) lf[a] = buf_ld<R>(plane_rsrc(li.f + a * pl, pbr), ocr);
    }
#pragma unroll
    for (int a = 0; a < 7; ++a) lg[a] = buf_ld<R>(plane_rsrc(li.g + a * pl, pbr), ocr);

    // ---- transposed enthalpy collision
    R Tb = 0, flb = 0, cpb = 0, sigb = 0, s6b = 0, uxb = 0, uyb = 0, uzb = 0;
    R lgo[7];
    if (MRT) {
      R r[7];
      mrt_rates(c, sig, r);
      const R qT = cp * T;
      // nu = N lg*, b_bar = -nu
      const R l12 = lg[1] + lg[2], l34 = lg[3] + lg[4], l56 = lg[5] + lg[6];
      const R bb1 = -(lg[1] - lg[2]), bb2 = -(lg[3] - lg[4]), bb3 = -(lg[5] - lg[6]);
      const R bb4 = -(static_cast<R>(6) * lg[0] - (l12 + l34 + l56));
      const R bb5 = -(static_cast<R>(2) * l12 - (l34 + l56));
      const R bb6 = -(l34 - l56);
      const R c1 = bb1 * r[1] * static_cast<R>(0.5), c2 = bb2 * r[2] * static_cast<R>(0.5),
              c3 = bb3 * r[3] * static_cast<R>(0.5);
      const R c4 = bb4 * r[4] * static_cast<R>(1.0 / 42.0);
      const R c5 = bb5 * r[5] * static_cast<R>(1.0 / 12.0);
      const R c6 = bb6 * r[6] * static_cast<R>(0.25);
      lgo[0] = lg[0];
      lgo[1] = lg[1] + c1 + static_cast<R>(2) * c5;
      lgo[2] = lg[2] - c1 + static_cast<R>(2) * c5;
      lgo[3] = lg[3] + c2 - c5 + c6;
      lgo[4] = lg[4] - c2 - c5 + c6;
      lgo[5] = lg[5] + c3 - c5 - c6;
      lgo[6] = lg[6] - c3 - c5 - c6;
      // q u terms
      const R qTb = -(c1 * ux + c2 * uy + c3 * uz);
      uxb += -c1 * qT;
      uyb += -c2 * qT;
      uzb += -c3 * qT;
      s6b += c4 * static_cast<R>(-7);
      Tb += c4 * static_cast<R>(21.0 * c.omega_T * c.cp_ref);
      cpb += qTb * T;
      Tb += qTb * cp;
      // rates
      const R g12 = g[1] + g[2], g34 = g[3] + g[4], g56 = g[5] + g[6];
      R rb[7];
      rb[1] = bb1 * (g[1] - g[2] - qT * ux) * static_cast<R>(0.5);
      rb[2] = bb2 * (g[3] - g[4] - qT * uy) * static_cast<R>(0.5);
      rb[3] = bb3 * (g[5] - g[6] - qT * uz) * static_cast<R>(0.5);
      rb[4] = bb4 * (static_cast<R>(-7) * s6 + static_cast<R>(21.0 * c.omega_T * c.cp_ref) * T) *
              static_cast<R>(1.0 / 42.0);
      rb[5] = bb5 * (static_cast<R>(2) * g12 - (g34 + g56)) * static_cast<R>(1.0 / 12.0);
      rb[6] = bb6 * (g34 - g56) * static_cast<R>(0.25);
#pragma unroll
      for (int k = 1; k < 7; ++k) {
        const bool fixed = c.has_override && !isnan(c.sig_ovr[k]);
        if (!fixed) sigb += k <= 3 ? rb[k] : -rb[k];
      }
    } else {
      const R it = sig;
      const R wT = static_cast<R>(0.5 * c.omega_T * c.cp_ref) * T;
      const R hq = static_cast<R>(0.5) * cp * T;
      lgo[0] = lg[0];
      Tb += -it * static_cast<R>(3.0 * c.omega_T * c.cp_ref) * lg[0];
      s6b += it * lg[0];
      sigb += -(static_cast<R>(3.0 * c.omega_T * c.cp_ref) * T - s6) * lg[0];
      R wTb = 0, hqb = 0;
#pragma unroll
      for (int a = 1; a < 7; ++a) {
        const R eu = Q7X[a] * ux + Q7Y[a] * uy + Q7Z[a] * uz;
        const R geq = wT + hq * eu;
        lgo[a] = lg[a] * (static_cast<R>(1) - it);
        wTb += it * lg[a];
        hqb += it * lg[a] * eu;
        const R e_hq = it * lg[a] * hq;
        uxb += Q7X[a] * e_hq;
        uyb += Q7Y[a] * e_hq;
        uzb += Q7Z[a] * e_hq;
        R ga = g[a];
        if constexpr (kShiftG<P>) ga += pars<R>(c).gshift;
        sigb += -(ga - geq) * lg[a];
      }
      Tb += static_cast<R>(0.5 * c.omega_T * c.cp_ref) * wTb + static_cast<R>(0.5) * cp * hqb;
      cpb += static_cast<R>(0.5) * T * hqb;
    }
    // sigma_chi(f_l) and C_p(f_l)
    flb += sigb * (-sig * sig * static_cast<R>(c.inv_rcw) * static_cast<R>(c.lam_l - c.lam_s));
    flb += cpb * static_cast<R>(c.cp_l - c.cp_s);

    // ---- transposed flow collision and forces
    if (FLOW) {
      R rb = 0, Fxb = 0, Fyb = 0, Fzb = 0, drb = 0;
      flow_collide_vjp<R>(c, lf, q, rb, uxb, uyb, uzb, Fxb, Fyb, Fzb, drb);
      // F = 2 (rho u - j0)
      rb += static_cast<R>(2) * (Fxb * ux + Fyb * uy + Fzb * uz);
      uxb += static_cast<R>(2) * q.rho * Fxb;
      uyb += static_cast<R>(2) * q.rho * Fyb;
      uzb += static_cast<R>(2) * q.rho * Fzb;
      R jxb = static_cast<R>(-2) * Fxb, jyb = static_cast<R>(-2) * Fyb, jz0b = static_cast<R>(-2) * Fzb;
      // u = f_l j / rho with jz = jz0 + F_b / 2
      const R irho = static_cast<R>(1) / q.rho;
      const R jz = q.jz0 + static_cast<R>(0.5) * static_cast<R>(c.g_beta_rho0) * (T - static_cast<R>(c.T_ref));
      jxb += uxb * fl * irho;
      jyb += uyb * fl * irho;
      const R jzb = uzb * fl * irho;
      flb += (uxb * q.jx + uyb * q.jy + uzb * jz) * irho;
      rb += -(uxb * ux + uyb * uy + uzb * uz) * irho;
      jz0b += jzb;
      Tb += static_cast<R>(0.5) * jzb * static_cast<R>(c.g_beta_rho0);
      drb += rb;
#pragma unroll
      for (int a = 0; a < 19; ++a) {
        R v = lf[a] + drb;
        if (Q19X[a] != 0) v += Q19X[a] > 0 ? jxb : -jxb;
        if (Q19Y[a] != 0) v += Q19Y[a] > 0 ? jyb : -jyb;
        if (Q19Z[a] != 0) v += Q19Z[a] > 0 ? jz0b : -jz0b;
        lf[a] = v;
      }
    }
    // ---- phase rule and h = sum g
    const R hb = Tb * dT_dh + flb * dfl_dh;
    lgo[0] = lgo[0] + hb;
#pragma unroll
    for (int a = 1; a < 7; ++a) lgo[a] = lgo[a] + hb + s6b;
    store_adjoint<R, FLOW>(c, make_site(c, cell), lo, pl, pbr, ocr, lf, lgo, dTw, last != 0);
  }
}

// Adjoint of the loss at the final state, lambda_g = seed dL/dh and
// lambda_f = 0, stored as M = S^T lambda_T for the last forward step (with
// its dL/dT_w contributions).
template <int P, bool FLOW>
__global__ void __launch_bounds__(256)
k_adj_seed(const CavParams* __restrict__ cavp, const char* __restrict__ state,
           char* __restrict__ lam, double scale, double* __restrict__ dTw) {
  using R = typename Fmt<P>::R;
  const CavParams& c = *cavp;
  const int32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= c.n) return;
  const int64_t pl = c.plane;
  const View<P> st = view<P>(state, c, FLOW);
  const AdjView<R> lv = adj_view<R>(lam, pl, FLOW);
  R g[7];
#pragma unroll
  for (int a = 1; a < 7; ++a) g[a] = dec(st.g[(a - 1) * pl + cell]);
  R s6 = moving_sum(g);
  if constexpr (kShiftG<P>) s6 += static_cast<R>(6) * pars<R>(c).gshift;
  const double h = load_g0<P>(st, cell) + static_cast<double>(s6);
  const double dfl = (h > c.hs && h < c.hl) ? c.inv_dh : 0.0;
  const R v = static_cast<R>(scale * dfl);
  R lf[19], lg[7];
#pragma unroll
  for (int a = 0; a < 19; ++a) lf[a] = 0;
#pragma unroll
  for (int a = 0; a < 7; ++a) lg[a] = v;
  const uint32_t pbr = static_cast<uint32_t>(pl) * static_cast<uint32_t>(sizeof(R));
  const uint32_t ocr = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(R));
  store_adjoint<R, FLOW>(c, make_site(c, cell), lv, pl, pbr, ocr, lf, lg, dTw, false);
}

// dL/dT0 from the adjoint of the initial state made by k_init: g_0 = h0 -
// 3 omega_T C_p,ref T0, g_a = (omega_T / 2) C_p,ref T0, dh0/dT0 = C_p of the
// phase of h0 (solid side at T0 = T_m).
template <int P, bool FLOW>
__global__ void __launch_bounds__(256)
k_adj_T0(const CavParams* __restrict__ cavp, const char* __restrict__ state0,
         const char* __restrict__ lam, double* __restrict__ out) {
  using R = typename Fmt<P>::R;
  const CavParams& c = *cavp;
  const int32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= c.n) return;
  const int64_t pl = c.plane;
  const View<P> st = view<P>(state0, c, FLOW);
  const AdjView<R> lv = adj_view<R>(lam, pl, FLOW);
  R g[7];
#pragma unroll
  for (int a = 1; a < 7; ++a) g[a] = dec(st.g[(a - 1) * pl + cell]);
  R s6 = moving_sum(g);
  if constexpr (kShiftG<P>) s6 += static_cast<R>(6) * pars<R>(c).gshift;
  const double h = load_g0<P>(st, cell) + static_cast<double>(s6);
  const double dh0 = h <= c.hs ? c.cp_s : c.cp_l;
  double s = 0.0;
#pragma unroll
  for (int a = 1; a < 7; ++a) s += static_cast<double>(lv.g[a * pl + cell]);
  out[cell] = static_cast<double>(lv.g[cell]) * (dh0 - 3.0 * c.omega_T * c.cp_ref) +
              0.5 * c.omega_T * c.cp_ref * s;
}

}  // namespace lbpc

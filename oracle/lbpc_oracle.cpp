// Plain FP64 CPU oracle for the coupled enthalpy / flow lattice Boltzmann step
// of Li & He, "Three-dimensional lattice Boltzmann models for solid-liquid phase
// change" (arXiv 1703.02652).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
// includes this file; only the tests, the smoke check and the CPU-baseline leg
// of the benchmark load it.  It shares no code, header or table with the HIP
// path.
//
// Style: slow and literal.  Dense transformation matrices typed in as printed
// (Eq. (24), Eq. (51)), inverted numerically; separate arrays for the pre- and
// post-collision states; one explicit branch per wall case.  Every function is
// a template on the scalar type so that a dual number (value, tangent) gives
// the exact discrete derivative of the step map (forward mode).  Branches are
// taken on the value part.
//
// Readings where the paper is silent, garbled or inconsistent are marked
// "reading:" in the comments below.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// --------------------------------------------------------------------------
// Scalars
// --------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double tan_part(double) { return 0.0; }
inline double tan_part(const Dual& x) { return x.d; }

// --------------------------------------------------------------------------
// Configuration (same field order as the cavity description dict)
// --------------------------------------------------------------------------
struct OrCfg {
  int32_t nx, ny, nz, flow, enth_model, precision;
  int32_t face_bc[6];
  double face_T[6];
  double omega_T, cp_s, cp_l, cp_ref, lambda_s, lambda_l, latent, T_m, rho0;
  double nu, s_e, s_eps, s_q, s_pi, s_t, g_beta, T_ref;
  double sigma_override[7];
};
enum { BC_PERIODIC = 0, BC_DIRICHLET = 1, BC_ADIABATIC = 2 };

// --------------------------------------------------------------------------
// Lattices
// --------------------------------------------------------------------------
// D3Q7 velocities, Eq. (3): rest, +x, -x, +y, -y, +z, -z.
const int E7[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                      {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
// D3Q7 moment matrix N, Eq. (24), as printed.
const int N7[7][7] = {
    {1, 1, 1, 1, 1, 1, 1},       {0, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0},      {0, 0, 0, 0, 0, 1, -1},
    {6, -1, -1, -1, -1, -1, -1}, {0, 2, 2, -1, -1, -1, -1},
    {0, 0, 0, 1, 1, -1, -1}};
// D3Q19 velocities, Eq. (48): columns of the printed 3 x 19 array.
const int E19[19][3] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
    {0, 0, 1},   {0, 0, -1},  {1, 1, 0},  {-1, 1, 0},  {1, -1, 0},
    {-1, -1, 0}, {1, 0, 1},   {-1, 0, 1}, {1, 0, -1},  {-1, 0, -1},
    {0, 1, 1},   {0, -1, 1},  {0, 1, -1}, {0, -1, -1}};
// D3Q19 moment matrix M, Eq. (51), as printed.
const int M19[19][19] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8},
    {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, -4, -4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, -2, -2, 2, 2, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1}};

// Numerical inverses of N and M (Gauss-Jordan with partial pivoting).
double N7inv[7][7];
double M19inv[19][19];
int OPP7[7], OPP19[19];

void invert(const double* a, double* out, int n) {
  std::vector<double> w(static_cast<size_t>(n) * 2 * n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) w[i * 2 * n + j] = a[i * n + j];
    w[i * 2 * n + n + i] = 1.0;
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(w[r * 2 * n + col]) > std::fabs(w[piv * 2 * n + col])) piv = r;
    if (piv != col)
      for (int j = 0; j < 2 * n; ++j) std::swap(w[col * 2 * n + j], w[piv * 2 * n + j]);
    const double p = w[col * 2 * n + col];
    for (int j = 0; j < 2 * n; ++j) w[col * 2 * n + j] /= p;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double fac = w[r * 2 * n + col];
      if (fac == 0.0) continue;
      for (int j = 0; j < 2 * n; ++j) w[r * 2 * n + j] -= fac * w[col * 2 * n + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[i * n + j] = w[i * 2 * n + n + j];
}

bool tables_ready = false;
void build_tables() {
  if (tables_ready) return;
  double a7[49], a19[361];
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 7; ++j) a7[i * 7 + j] = N7[i][j];
  for (int i = 0; i < 19; ++i)
    for (int j = 0; j < 19; ++j) a19[i * 19 + j] = M19[i][j];
  invert(a7, &N7inv[0][0], 7);
  invert(a19, &M19inv[0][0], 19);
  for (int a = 0; a < 7; ++a)
    for (int b = 0; b < 7; ++b)
      if (E7[b][0] == -E7[a][0] && E7[b][1] == -E7[a][1] && E7[b][2] == -E7[a][2])
        OPP7[a] = b;
  for (int a = 0; a < 19; ++a)
    for (int b = 0; b < 19; ++b)
      if (E19[b][0] == -E19[a][0] && E19[b][1] == -E19[a][1] && E19[b][2] == -E19[a][2])
        OPP19[a] = b;
  tables_ready = true;
}

// D3Q7 weights, Eq. (8).
double w7(const OrCfg& c, int a) { return a == 0 ? 1.0 - 3.0 * c.omega_T : 0.5 * c.omega_T; }

// --------------------------------------------------------------------------
// Macroscopic relations
// --------------------------------------------------------------------------
// Enthalpy -> (T, f_l), Eq. (2) with h0 = 0.  Reading: the inverse is the
// lever rule, isothermal at T_m across the mushy range; h_s = C_p,s T_m and
// h_l = C_p,l T_m + L; closed toward the pure phases.
template <class S>
void phase(const OrCfg& c, S h, S& T, S& fl) {
  const double hs = c.cp_s * c.T_m;
  const double hl = c.cp_l * c.T_m + c.latent;
  if (val(h) <= hs) {
    fl = S(0.0);
    T = h / S(c.cp_s);
  } else if (val(h) >= hl) {
    fl = S(1.0);
    T = (h - S(c.latent)) / S(c.cp_l);
  } else {
    fl = (h - S(hs)) / S(hl - hs);
    T = S(c.T_m);
  }
}

// Local specific heat and conductivity: linear mixture in f_l.
template <class S> S mix(S fl, double a_s, double a_l) { return S(a_s) + fl * S(a_l - a_s); }

// tau_g from Eq. (20) with chi = lambda / (rho0 C_p,ref) (Eq. (19) vs Eq. (1)).
template <class S> S tau_g(const OrCfg& c, S lam) {
  return lam / S(c.rho0 * c.cp_ref * c.omega_T) + S(0.5);
}

// Equilibrium of the enthalpy distribution, Eq. (7).
template <class S>
void g_eq(const OrCfg& c, S h, S T, S cp, const S u[3], S geq[7]) {
  geq[0] = h - S(1.0 - w7(c, 0)) * S(c.cp_ref) * T;
  for (int a = 1; a < 7; ++a) {
    S eu = u[0] * S(E7[a][0]) + u[1] * S(E7[a][1]) + u[2] * S(E7[a][2]);
    geq[a] = S(w7(c, a) * c.cp_ref) * T + eu / S(c.omega_T) * S(w7(c, a)) * cp * T;
  }
}

// Equilibrium moments of the enthalpy distribution, Eq. (25) (c = 1).
template <class S>
void n_eq(const OrCfg& c, S h, S T, S cp, const S u[3], S neq[7]) {
  neq[0] = h;
  neq[1] = cp * T * u[0];
  neq[2] = cp * T * u[1];
  neq[3] = cp * T * u[2];
  neq[4] = S(6.0) * h - S(21.0 * c.omega_T * c.cp_ref) * T;
  neq[5] = S(0.0);
  neq[6] = S(0.0);
}

// Equilibrium moments of the flow distribution, Eq. (53) (c = 1).
// Reading: the printed 11th entry, -u_x^2 + 0.5 u_y^2 + u_z^2, is taken as
// -u_x^2 + u_y^2/2 + u_z^2/2, i.e. -1/2 of the 10th entry, as for the other
// pi-type moment in the same line.
template <class S>
void m_eq(S rho, const S u[3], S meq[19]) {
  const S ux = u[0], uy = u[1], uz = u[2];
  const S u2 = ux * ux + uy * uy + uz * uz;
  meq[0] = rho;
  meq[1] = rho * (S(-11.0) + S(19.0) * u2);
  meq[2] = rho * (S(3.0) - S(11.0 / 2.0) * u2);
  meq[3] = rho * ux;
  meq[4] = rho * S(-2.0 / 3.0) * ux;
  meq[5] = rho * uy;
  meq[6] = rho * S(-2.0 / 3.0) * uy;
  meq[7] = rho * uz;
  meq[8] = rho * S(-2.0 / 3.0) * uz;
  meq[9] = rho * (S(3.0) * ux * ux - u2);
  meq[10] = rho * (-ux * ux + S(0.5) * uy * uy + S(0.5) * uz * uz);
  meq[11] = rho * (uy * uy - uz * uz);
  meq[12] = rho * (uz * uz - uy * uy) / S(2.0);
  meq[13] = rho * ux * uy;
  meq[14] = rho * uy * uz;
  meq[15] = rho * uz * ux;
  meq[16] = S(0.0);
  meq[17] = S(0.0);
  meq[18] = S(0.0);
}

// Forcing moments, Eq. (54) (c = 1).
// Reading: the printed 10th entry, 2 F_x u_x - 2 F.u, is taken as
// 6 F_x u_x - 2 F.u, i.e. -2 times the 11th entry, as for the other pair.
template <class S>
void force_moments(const S F[3], const S u[3], S ff[19]) {
  const S Fu = F[0] * u[0] + F[1] * u[1] + F[2] * u[2];
  ff[0] = S(0.0);
  ff[1] = S(38.0) * Fu;
  ff[2] = S(-11.0) * Fu;
  ff[3] = F[0];
  ff[4] = S(-2.0 / 3.0) * F[0];
  ff[5] = F[1];
  ff[6] = S(-2.0 / 3.0) * F[1];
  ff[7] = F[2];
  ff[8] = S(-2.0 / 3.0) * F[2];
  ff[9] = S(6.0) * F[0] * u[0] - S(2.0) * Fu;
  ff[10] = Fu - S(3.0) * F[0] * u[0];
  ff[11] = S(2.0) * F[1] * u[1] - S(2.0) * F[2] * u[2];
  ff[12] = F[2] * u[2] - F[1] * u[1];
  ff[13] = F[0] * u[1] + F[1] * u[0];
  ff[14] = F[1] * u[2] + F[2] * u[1];
  ff[15] = F[0] * u[2] + F[2] * u[0];
  ff[16] = S(0.0);
  ff[17] = S(0.0);
  ff[18] = S(0.0);
}

// Diagonal of the flow relaxation matrix, Eq. (52); s_nu from Eq. (59).
void flow_rates(const OrCfg& c, double lam[19]) {
  const double s_nu = 1.0 / (3.0 * c.nu + 0.5);
  const double d[19] = {0.0,  c.s_e,  c.s_eps, 0.0,  c.s_q, 0.0,  c.s_q,
                        0.0,  c.s_q,  s_nu,    c.s_pi, s_nu, c.s_pi, s_nu,
                        s_nu, s_nu,   c.s_t,   c.s_t, c.s_t};
  for (int k = 0; k < 19; ++k) lam[k] = d[k];
}

// --------------------------------------------------------------------------
// One cell: macroscopic update, both collisions.
// --------------------------------------------------------------------------
template <class S> struct CellOut {
  S h, T, fl, cp, rho, u[3], F[3];
};

// Flow part of a cell (Sec. 2.5).  Reading of "solid-region forcing" and of
// buoyancy "in the liquid phase domain": the velocity is u = f_l j / rho with
// j = sum f e + F_b / 2, and the total force F = 2 (rho u - sum f e) makes
// Eq. (56) hold with the local density; u = 0 in solid cells, F = F_b in
// liquid ones.  Buoyancy Eq. (55) with rho_ref = rho0.
template <class S>
void flow_collide(const OrCfg& c, const S f[19], S T, S fl, S fs[19], CellOut<S>& o) {
  S rho = S(0.0), mom[3] = {S(0.0), S(0.0), S(0.0)};
  for (int a = 0; a < 19; ++a) {
    rho += f[a];
    for (int d = 0; d < 3; ++d) mom[d] += f[a] * S(E19[a][d]);
  }
  S Fb[3] = {S(0.0), S(0.0), S(c.g_beta * c.rho0) * (T - S(c.T_ref))};
  S u[3], F[3];
  for (int d = 0; d < 3; ++d) {
    S j = mom[d] + Fb[d] / S(2.0);
    u[d] = fl * j / rho;
    F[d] = S(2.0) * (rho * u[d] - mom[d]);
  }
  S m[19];
  for (int k = 0; k < 19; ++k) {
    m[k] = S(0.0);
    for (int a = 0; a < 19; ++a) m[k] += S(M19[k][a]) * f[a];
  }
  S meq[19], ff[19];
  m_eq(rho, u, meq);
  force_moments(F, u, ff);
  double lam[19];
  flow_rates(c, lam);
  S mpost[19];
  for (int k = 0; k < 19; ++k)  // Eq. (49), delta_t = 1
    mpost[k] = m[k] - S(lam[k]) * (m[k] - meq[k]) + S(1.0 - 0.5 * lam[k]) * ff[k];
  for (int a = 0; a < 19; ++a) {  // Eq. (50): back to velocity space
    fs[a] = S(0.0);
    for (int k = 0; k < 19; ++k) fs[a] += S(M19inv[a][k]) * mpost[k];
  }
  o.rho = rho;
  for (int d = 0; d < 3; ++d) {
    o.u[d] = u[d];
    o.F[d] = F[d];
  }
}

// Enthalpy part of a cell (Sec. 2.2 SRT, Sec. 2.3 MRT).
// Reading of the relaxation set: sigma_1..3 = sigma_chi = 1 / tau_g (Eq. (23),
// (34)); sigma_4..6 = 2 - sigma_chi (the rule of Eq. (47), with sigma_4 =
// sigma_5 as used in Sec. 3.1.2, extended to sigma_6 so that y and z links
// cancel the interface error as x links do); sigma_0 = sigma_chi (it multiplies
// n_0 - n_0^eq = 0).  A finite entry of sigma_override replaces that rate.
template <class S>
void enthalpy_collide(const OrCfg& c, const S g[7], S h, S T, S fl, S cp, const S u[3],
                      S gs[7]) {
  const S lam = mix(fl, c.lambda_s, c.lambda_l);
  const S tau = tau_g(c, lam);
  if (c.enth_model == 0) {  // SRT, Eq. (5)-(7)
    S geq[7];
    g_eq(c, h, T, cp, u, geq);
    for (int a = 0; a < 7; ++a) gs[a] = g[a] - (g[a] - geq[a]) / tau;
    return;
  }
  const S sig_chi = S(1.0) / tau;
  S R[7] = {sig_chi, sig_chi, sig_chi, sig_chi, S(2.0) - sig_chi, S(2.0) - sig_chi,
            S(2.0) - sig_chi};
  for (int k = 0; k < 7; ++k)
    if (!std::isnan(c.sigma_override[k])) R[k] = S(c.sigma_override[k]);
  S n[7], neq[7], npost[7];
  for (int k = 0; k < 7; ++k) {
    n[k] = S(0.0);
    for (int a = 0; a < 7; ++a) n[k] += S(N7[k][a]) * g[a];
  }
  n_eq(c, h, T, cp, u, neq);
  for (int k = 0; k < 7; ++k) npost[k] = n[k] - R[k] * (n[k] - neq[k]);  // Eq. (21)
  for (int a = 0; a < 7; ++a) {
    gs[a] = S(0.0);
    for (int k = 0; k < 7; ++k) gs[a] += S(N7inv[a][k]) * npost[k];
  }
}

// Full cell update.  Reading of the coupling order: both collisions use the
// macroscopic fields of the same (pre-collision) time level.
template <class S>
void collide_cell(const OrCfg& c, const S* f, const S g[7], S* fs, S gs[7], CellOut<S>& o) {
  S h = S(0.0);
  for (int a = 0; a < 7; ++a) h += g[a];
  S T, fl;
  phase(c, h, T, fl);
  const S cp = mix(fl, c.cp_s, c.cp_l);
  o.h = h;
  o.T = T;
  o.fl = fl;
  o.cp = cp;
  o.rho = S(0.0);
  for (int d = 0; d < 3; ++d) o.u[d] = o.F[d] = S(0.0);
  if (c.flow) flow_collide(c, f, T, fl, fs, o);
  enthalpy_collide(c, g, h, T, fl, cp, o.u, gs);
}

// --------------------------------------------------------------------------
// Lattice
// --------------------------------------------------------------------------
struct Grid {
  int nx, ny, nz;
  int64_t n;
  int64_t idx(int x, int y, int z) const { return x + (int64_t)nx * (y + (int64_t)ny * z); }
};

// Offsets of each face's node field inside the concatenated wall array:
// x faces [nz][ny], y faces [nz][nx], z faces [ny][nx].
void face_offsets(const Grid& G, int64_t off[7]) {
  const int64_t sz[6] = {(int64_t)G.ny * G.nz, (int64_t)G.ny * G.nz, (int64_t)G.nx * G.nz,
                         (int64_t)G.nx * G.nz, (int64_t)G.nx * G.ny, (int64_t)G.nx * G.ny};
  off[0] = 0;
  for (int i = 0; i < 6; ++i) off[i + 1] = off[i] + sz[i];
}
int64_t face_node(const Grid& G, int face, int x, int y, int z) {
  const int dim = face / 2;
  if (dim == 0) return y + (int64_t)G.ny * z;
  if (dim == 1) return x + (int64_t)G.nx * z;
  return x + (int64_t)G.nx * y;
}

// Streaming, pull form of Eq. (5) and Eq. (50): the population moving along e_a
// arriving at x left x - e_a.  Reading of the walls (half a cell outside the
// first and last nodes): a link that leaves the lattice through a non-periodic
// face comes back to its own node reversed; for f always (no-slip, halfway
// bounce-back); for g plain reflection on adiabatic faces and, on fixed-
// temperature faces, g_a(x) = -g*_abar(x) + 2 w_a C_p,ref T_w (anti-bounce-back).
// Returns, for budgets, the enthalpy that entered through the walls.
template <class S>
S stream(const OrCfg& c, const Grid& G, const S* fs, const S* gs, S* f, S* g, const S* tw) {
  int64_t foff[7];
  face_offsets(G, foff);
  const int dims[3] = {G.nx, G.ny, G.nz};
  std::vector<S> plane_flux(G.nz, S(0.0));
#pragma omp parallel for schedule(static)
  for (int z = 0; z < G.nz; ++z) {
    S flux = S(0.0);
      for (int y = 0; y < G.ny; ++y)
        for (int x = 0; x < G.nx; ++x) {
          const int64_t i = G.idx(x, y, z);
          const int p[3] = {x, y, z};
          if (c.flow) {
            for (int a = 0; a < 19; ++a) {
              int q[3];
              bool wall = false;
              for (int d = 0; d < 3; ++d) {
                q[d] = p[d] - E19[a][d];
                if (q[d] < 0 || q[d] >= dims[d]) {
                  if (c.face_bc[2 * d] == BC_PERIODIC) q[d] = (q[d] + dims[d]) % dims[d];
                  else wall = true;
                }
              }
              if (wall) f[i * 19 + a] = fs[i * 19 + OPP19[a]];
              else f[i * 19 + a] = fs[G.idx(q[0], q[1], q[2]) * 19 + a];
            }
          }
          for (int a = 0; a < 7; ++a) {
            int q[3];
            int face = -1;
            for (int d = 0; d < 3; ++d) {
              q[d] = p[d] - E7[a][d];
              if (q[d] < 0 || q[d] >= dims[d]) {
                if (c.face_bc[2 * d] == BC_PERIODIC) q[d] = (q[d] + dims[d]) % dims[d];
                else face = 2 * d + (q[d] < 0 ? 0 : 1);
              }
            }
            if (face < 0) {
              g[i * 7 + a] = gs[G.idx(q[0], q[1], q[2]) * 7 + a];
            } else if (c.face_bc[face] == BC_ADIABATIC) {
              g[i * 7 + a] = gs[i * 7 + OPP7[a]];
            } else {  // BC_DIRICHLET
              const S Tw = tw[foff[face] + face_node(G, face, x, y, z)];
              const S in = -gs[i * 7 + OPP7[a]] + S(2.0 * w7(c, a) * c.cp_ref) * Tw;
              g[i * 7 + a] = in;
              flux += in - gs[i * 7 + OPP7[a]];
            }
          }
        }
    plane_flux[z] = flux;
  }
  S flux_total = S(0.0);
  for (int z = 0; z < G.nz; ++z) flux_total += plane_flux[z];
  return flux_total;
}

template <class S> struct Budget {
  S H, mass, fl, flux;
};

// One time step on the whole lattice: collide every cell, then stream.
template <class S>
Budget<S> step(const OrCfg& c, const Grid& G, S* f, S* g, S* fs, S* gs, const S* tw) {
  std::vector<S> hrow(G.nz), mrow(G.nz), frow(G.nz);
#pragma omp parallel for schedule(static)
  for (int z = 0; z < G.nz; ++z) {
    S hz = S(0.0), mz = S(0.0), fz = S(0.0);
    for (int y = 0; y < G.ny; ++y)
      for (int x = 0; x < G.nx; ++x) {
        const int64_t i = G.idx(x, y, z);
        CellOut<S> o;
        collide_cell(c, c.flow ? f + i * 19 : nullptr, g + i * 7,
                     c.flow ? fs + i * 19 : nullptr, gs + i * 7, o);
        hz += o.h;
        mz += o.rho;
        fz += o.fl;
      }
    hrow[z] = hz;
    mrow[z] = mz;
    frow[z] = fz;
  }
  Budget<S> b;
  b.H = b.mass = b.fl = S(0.0);
  for (int z = 0; z < G.nz; ++z) {
    b.H += hrow[z];
    b.mass += mrow[z];
    b.fl += frow[z];
  }
  b.flux = stream(c, G, fs, gs, f, g, tw);
  return b;
}

Grid grid_of(const OrCfg* c) {
  Grid G;
  G.nx = c->nx;
  G.ny = c->ny;
  G.nz = c->nz;
  G.n = (int64_t)c->nx * c->ny * c->nz;
  return G;
}

int64_t wall_len(const Grid& G) {
  int64_t off[7];
  face_offsets(G, off);
  return off[6];
}

// Initial state.  Flow at rest: f = M^-1 m^eq(rho0, 0).  Enthalpy at rest:
// g = g^eq(h0(T0), T0, u = 0) with h0 from Eq. (2): solid (T0 <= T_m, f_l = 0)
// h0 = C_p,s T0, liquid h0 = C_p,l T0 + L (reading: T0 = T_m is solid).
template <class S>
void init_cell(const OrCfg& c, S T0, S* f, S g[7]) {
  if (c.flow && f) {
    S meq[19], u0[3] = {S(0.0), S(0.0), S(0.0)};
    m_eq(S(c.rho0), u0, meq);
    for (int a = 0; a < 19; ++a) {
      f[a] = S(0.0);
      for (int k = 0; k < 19; ++k) f[a] += S(M19inv[a][k]) * meq[k];
    }
  }
  S h0, cp;
  if (val(T0) <= c.T_m) {
    h0 = S(c.cp_s) * T0;
    cp = S(c.cp_s);
  } else {
    h0 = S(c.cp_l) * T0 + S(c.latent);
    cp = S(c.cp_l);
  }
  S u0[3] = {S(0.0), S(0.0), S(0.0)};
  g_eq(c, h0, T0, cp, u0, g);
}

template <class S>
S loss_of(const OrCfg& c, const Grid& G, const S* g, int kind) {
  std::vector<S> row(G.nz);
#pragma omp parallel for schedule(static)
  for (int z = 0; z < G.nz; ++z) {
    S acc = S(0.0);
    for (int y = 0; y < G.ny; ++y)
      for (int x = 0; x < G.nx; ++x) {
        const int64_t i = G.idx(x, y, z);
        S h = S(0.0);
        for (int a = 0; a < 7; ++a) h += g[i * 7 + a];
        S T, fl;
        phase(c, h, T, fl);
        acc += fl;
      }
    row[z] = acc;
  }
  S L = S(0.0);
  for (int z = 0; z < G.nz; ++z) L += row[z];
  if (kind == 1) L = L / S((double)G.ny * G.nz);
  return L;
}

}  // namespace

// --------------------------------------------------------------------------
// C interface (ctypes).  State arrays are cell-major: f[cell*19 + a], g[cell*7 + a],
// cell = x + nx*(y + ny*z).
// --------------------------------------------------------------------------
extern "C" {

int or_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads for the following runs (timing on one core against all cores).
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

void or_tables(double* e7, double* e19, double* n7, double* n7inv, double* m19,
               double* m19inv) {
  build_tables();
  for (int a = 0; a < 7; ++a)
    for (int d = 0; d < 3; ++d) e7[a * 3 + d] = E7[a][d];
  for (int a = 0; a < 19; ++a)
    for (int d = 0; d < 3; ++d) e19[a * 3 + d] = E19[a][d];
  for (int i = 0; i < 49; ++i) {
    n7[i] = N7[i / 7][i % 7];
    n7inv[i] = N7inv[i / 7][i % 7];
  }
  for (int i = 0; i < 361; ++i) {
    m19[i] = M19[i / 19][i % 19];
    m19inv[i] = M19inv[i / 19][i % 19];
  }
}

void or_g_eq(const OrCfg* c, double h, double T, double cp, const double* u, double* out) {
  build_tables();
  g_eq<double>(*c, h, T, cp, u, out);
}
void or_n_eq(const OrCfg* c, double h, double T, double cp, const double* u, double* out) {
  build_tables();
  n_eq<double>(*c, h, T, cp, u, out);
}
void or_m_eq(double rho, const double* u, double* out) { m_eq<double>(rho, u, out); }
void or_force_moments(const double* F, const double* u, double* out) {
  force_moments<double>(F, u, out);
}
void or_phase(const OrCfg* c, double h, double* T, double* fl) { phase<double>(*c, h, *T, *fl); }

// aux: h, T, f_l, C_p, rho, u[3], F[3]
void or_collide_cell(const OrCfg* c, const double* f, const double* g, double* fs,
                     double* gs, double* aux) {
  build_tables();
  CellOut<double> o;
  collide_cell<double>(*c, f, g, fs, gs, o);
  if (aux) {
    const double v[11] = {o.h, o.T, o.fl, o.cp, o.rho, o.u[0], o.u[1], o.u[2],
                          o.F[0], o.F[1], o.F[2]};
    std::memcpy(aux, v, sizeof(v));
  }
}

int or_init(const OrCfg* c, const double* T0, double* f, double* g) {
  build_tables();
  const Grid G = grid_of(c);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < G.n; ++i)
    init_cell<double>(*c, T0 ? T0[i] : c->T_m, c->flow ? f + i * 19 : nullptr, g + i * 7);
  return 0;
}

// hist (nullable): per step H, mass, sum f_l (pre-collision) and the wall flux.
int or_run(const OrCfg* c, double* f, double* g, const double* tw, int64_t nsteps,
           double* hist) {
  build_tables();
  const Grid G = grid_of(c);
  std::vector<double> fs(c->flow ? G.n * 19 : 0), gs(G.n * 7);
  for (int64_t t = 0; t < nsteps; ++t) {
    Budget<double> b = step<double>(*c, G, f, g, c->flow ? fs.data() : nullptr, gs.data(), tw);
    if (hist) {
      hist[4 * t + 0] = b.H;
      hist[4 * t + 1] = b.mass;
      hist[4 * t + 2] = b.fl;
      hist[4 * t + 3] = b.flux;
    }
  }
  return 0;
}

// out per cell: h, T, f_l, rho, u_x, u_y, u_z  (u from Eq. (56) with the forcing)
int or_fields(const OrCfg* c, const double* f, const double* g, double* out) {
  build_tables();
  const Grid G = grid_of(c);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < G.n; ++i) {
    double fsc[19], gsc[7];
    CellOut<double> o;
    collide_cell<double>(*c, c->flow ? f + i * 19 : nullptr, g + i * 7,
                         c->flow ? fsc : nullptr, gsc, o);
    out[i * 7 + 0] = o.h;
    out[i * 7 + 1] = o.T;
    out[i * 7 + 2] = o.fl;
    out[i * 7 + 3] = o.rho;
    out[i * 7 + 4] = o.u[0];
    out[i * 7 + 5] = o.u[1];
    out[i * 7 + 6] = o.u[2];
  }
  return 0;
}

double or_loss(const OrCfg* c, const double* g, int kind) {
  build_tables();
  return loss_of<double>(*c, grid_of(c), g, kind);
}

// Tangent of the loss after nsteps along a direction in (initial state, wall
// temperatures).  df, dg, dtw may be null (zero direction).
int or_run_tangent(const OrCfg* c, const double* f, const double* g, const double* df,
                   const double* dg, const double* tw, const double* dtw, int64_t nsteps,
                   int loss_kind, double* loss, double* dloss) {
  build_tables();
  const Grid G = grid_of(c);
  const int64_t nf = c->flow ? G.n * 19 : 0, ng = G.n * 7, nw = wall_len(G);
  std::vector<Dual> F(nf), Gd(ng), Fs(nf), Gs(ng), TW(nw);
  for (int64_t i = 0; i < nf; ++i) F[i] = Dual(f[i], df ? df[i] : 0.0);
  for (int64_t i = 0; i < ng; ++i) Gd[i] = Dual(g[i], dg ? dg[i] : 0.0);
  for (int64_t i = 0; i < nw; ++i) TW[i] = Dual(tw[i], dtw ? dtw[i] : 0.0);
  for (int64_t t = 0; t < nsteps; ++t)
    step<Dual>(*c, G, c->flow ? F.data() : nullptr, Gd.data(), c->flow ? Fs.data() : nullptr,
               Gs.data(), TW.data());
  const Dual L = loss_of<Dual>(*c, G, Gd.data(), loss_kind);
  *loss = L.v;
  *dloss = L.d;
  return 0;
}

// Tangent of the initial state along a direction dT0 of the initial temperature.
int or_init_tangent(const OrCfg* c, const double* T0, const double* dT0, double* f,
                    double* g, double* df, double* dg) {
  build_tables();
  const Grid G = grid_of(c);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < G.n; ++i) {
    Dual fd[19], gd[7];
    init_cell<Dual>(*c, Dual(T0 ? T0[i] : c->T_m, dT0 ? dT0[i] : 0.0),
                    c->flow ? fd : nullptr, gd);
    if (c->flow)
      for (int a = 0; a < 19; ++a) {
        f[i * 19 + a] = fd[a].v;
        df[i * 19 + a] = fd[a].d;
      }
    for (int a = 0; a < 7; ++a) {
      g[i * 7 + a] = gd[a].v;
      dg[i * 7 + a] = gd[a].d;
    }
  }
  return 0;
}

}  // extern "C"

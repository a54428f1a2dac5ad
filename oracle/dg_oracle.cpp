// dg_oracle.cpp -- serial FP64 reference implementation of the DGSEM residual.
//
// TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the HIP
// path is checked.  Only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark may load it.  It shares no code, header, table or
// helper with the GPU library, and it is deliberately plain: loops over
// elements, sides and nodes in the order the equations are written, no
// blocking, no fusion.
//
// What it computes (paper: "Governing Equations and Numerical Method"):
//   * compressible Euler / Navier-Stokes-Fourier fluxes, perfect gas
//     (the caloric EOS is read as p = (gamma-1) rho eps; the printed sign is
//     garbled);
//   * the collocated DGSEM weak form, eq. (dgsem_weak), on LG or LGL nodes;
//   * BR1 lifting of the primitive gradients (u,v,w,T), eq. (dgsem_lifted),
//     with the central face average;
//   * the split-form (flux-differencing) volume integral with the
//     Chandrashekar kinetic-energy-preserving, entropy-conservative two-point
//     flux on LGL nodes;
//   * its entropy-stable counterpart on LG nodes (the configuration of the
//     paper's TGV and PID comparisons, which it attributes to Schwarz et al.
//     2025 without stating the scheme): read here as the hybridised SBP
//     operator with entropy projection of Chan, Del Rey Fernandez & Carpenter
//     (SISC 2019), written out literally per line (hybrid_line);
//   * the Rusanov surface flux (the paper's Roe flux is a later addition);
//     the viscous surface flux is the arithmetic mean of both sides;
//   * the low-storage RK4(5) scheme of Carpenter and Kennedy;
//   * the integral kinetic energy E_k (TGV section) and its gradient;
//   * forward-mode tangents (dual numbers) of the residual and of whole RK
//     trajectories;
//   * reverse mode: the transposed residual Jacobian applied to a vector
//     (a taped scalar swept backwards), the gradient of E_k, and the reverse
//     sweep of the 2N-storage RK stages over a whole trajectory (the
//     adjoint the GPU path is checked against; not in the paper);
//   * operation counts of the residual as written (a counting scalar).
//
// Function pins (closed forms, invariants, brute force) live in tests/.
// Everything with no such pin is listed as "parity unpinned" below:
//   * (none: every exported routine has at least one pin in tests/)
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>
#include <array>

namespace orc {

// ---------------------------------------------------------------------------
// Scalar types.  The residual is written once as a template and evaluated
// with plain doubles, with dual numbers (exact directional derivatives), with
// a taped reverse-mode scalar (exact transposed products) and with an
// operation-counting double.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, a.d * e); }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline double val(Dual a) { return a.v; }
inline double val(double a) { return a; }

// Operation counter: each +,-,* ,/, sqrt, log on a Cnt bumps a counter.
struct Cnt {
  double v;
  Cnt(double a = 0.0) : v(a) {}
  static uint64_t n_add, n_mul, n_div, n_sqrt, n_log;
};
uint64_t Cnt::n_add = 0, Cnt::n_mul = 0, Cnt::n_div = 0, Cnt::n_sqrt = 0, Cnt::n_log = 0;
inline Cnt operator+(Cnt a, Cnt b) { ++Cnt::n_add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++Cnt::n_add; return Cnt(a.v - b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++Cnt::n_mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++Cnt::n_div; return Cnt(a.v / b.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, Cnt b) { a = a * b; return a; }
inline Cnt log(Cnt a) { ++Cnt::n_log; return Cnt(std::log(a.v)); }
inline Cnt exp(Cnt a) { ++Cnt::n_log; return Cnt(std::exp(a.v)); }   // counted with log
inline Cnt sqrt(Cnt a) { ++Cnt::n_sqrt; return Cnt(std::sqrt(a.v)); }
inline double val(Cnt a) { return a.v; }

// Reverse-mode scalar.  Every operation on a Rev whose operands depend on the
// inputs appends one node to the tape: the indices of its (at most two)
// operand nodes and the partial derivatives with respect to them.  Sweeping
// the tape from the end with the outputs' adjoints as seeds gives the
// vector-Jacobian product (dY/dX)^T lam exactly (up to rounding): the
// transposed chain rule applied operation by operation.  Operations on
// constants (node index -1) are not recorded.
struct Tape {
  struct Node {
    int a, b;        // operand nodes (-1: none)
    double da, db;   // partial derivatives with respect to them
  };
  std::vector<Node> nodes;
  int push(int a, double da, int b, double db) {
    nodes.push_back(Node{a, b, da, db});
    return (int)nodes.size() - 1;
  }
  void clear() { nodes.clear(); }
  size_t size() const { return nodes.size(); }
  // adj holds one adjoint per node (seeded at the outputs); on return the
  // adjoints of all nodes, in particular of the independent variables.
  void sweep(std::vector<double>& adj) const {
    for (size_t n = nodes.size(); n-- > 0;) {
      const double x = adj[n];
      if (x == 0.0) continue;
      const Node& d = nodes[n];
      if (d.a >= 0) adj[d.a] += d.da * x;
      if (d.b >= 0) adj[d.b] += d.db * x;
    }
  }
};
static Tape g_tape;

struct Rev {
  double v;
  int i;   // tape node, -1 for a constant
  Rev(double a = 0.0) : v(a), i(-1) {}
  Rev(double a, int node) : v(a), i(node) {}
  static Rev input(double a) { return Rev(a, g_tape.push(-1, 0.0, -1, 0.0)); }
};
inline Rev rev_node(double v, int a, double da, int b, double db) {
  if (a < 0 && b < 0) return Rev(v);
  return Rev(v, g_tape.push(a, da, b, db));
}
inline Rev operator+(Rev a, Rev b) { return rev_node(a.v + b.v, a.i, 1.0, b.i, 1.0); }
inline Rev operator-(Rev a, Rev b) { return rev_node(a.v - b.v, a.i, 1.0, b.i, -1.0); }
inline Rev operator-(Rev a) { return rev_node(-a.v, a.i, -1.0, -1, 0.0); }
inline Rev operator*(Rev a, Rev b) { return rev_node(a.v * b.v, a.i, b.v, b.i, a.v); }
inline Rev operator/(Rev a, Rev b) {
  const double q = a.v / b.v;
  return rev_node(q, a.i, 1.0 / b.v, b.i, -q / b.v);
}
inline Rev& operator+=(Rev& a, Rev b) { a = a + b; return a; }
inline Rev& operator-=(Rev& a, Rev b) { a = a - b; return a; }
inline Rev& operator*=(Rev& a, Rev b) { a = a * b; return a; }
inline Rev log(Rev a) { return rev_node(std::log(a.v), a.i, 1.0 / a.v, -1, 0.0); }
inline Rev exp(Rev a) { const double e = std::exp(a.v); return rev_node(e, a.i, e, -1, 0.0); }
inline Rev sqrt(Rev a) { const double r = std::sqrt(a.v); return rev_node(r, a.i, 0.5 / r, -1, 0.0); }
inline double val(Rev a) { return a.v; }

using std::log;
using std::exp;
using std::sqrt;

// max that keeps the first argument on ties; |x| by sign of the value.
template <class T> inline T maxv(const T& a, const T& b) { return val(a) >= val(b) ? a : b; }
template <class T> inline T absv(const T& a) { return val(a) >= 0.0 ? a : T(-a); }

// ---------------------------------------------------------------------------
// 1-D basis (Kopriva, "Implementing Spectral Methods for PDEs", Legendre node
// algorithms): nodes, weights, differentiation matrix, boundary values.
// ---------------------------------------------------------------------------
static void legendre(int n, double x, double& P, double& dP) {
  // Three-term recurrence for P_n and its derivative.
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  if (n == 1) { P = x; dP = 1.0; return; }
  double Pm2 = 1.0, Pm1 = x, dPm2 = 0.0, dPm1 = 1.0, Pk = 0.0, dPk = 0.0;
  for (int k = 2; k <= n; ++k) {
    Pk = ((2.0 * k - 1.0) * x * Pm1 - (k - 1.0) * Pm2) / k;
    dPk = dPm2 + (2.0 * k - 1.0) * Pm1;
    Pm2 = Pm1; Pm1 = Pk; dPm2 = dPm1; dPm1 = dPk;
  }
  P = Pk; dP = dPk;
}

struct Basis {
  int N = 0, type = 0;          // type 0 = Legendre-Gauss, 1 = Legendre-Gauss-Lobatto
  std::vector<double> x, w;     // nodes and quadrature weights
  std::vector<double> D;        // D[i*(N+1)+j] = l_j'(x_i)
  std::vector<double> Lm, Lp;   // l_j(-1), l_j(+1)
  std::vector<double> DS;       // split operator 2D - e_N e_N^T/w_N + e_0 e_0^T/w_0 (LGL)
};

static bool make_basis(int N, int type, Basis& B) {
  if (N < 1 || N > 15 || (type != 0 && type != 1)) return false;
  const int n = N + 1;
  B.N = N; B.type = type;
  B.x.assign(n, 0.0); B.w.assign(n, 0.0);
  const double pi = std::acos(-1.0);
  if (type == 0) {
    // Roots of P_{N+1}; weights 2 / ((1-x^2) P'_{N+1}(x)^2).
    for (int j = 0; j < n; ++j) {
      double xj = -std::cos((2.0 * j + 1.0) * pi / (2.0 * N + 2.0));
      for (int it = 0; it < 100; ++it) {
        double P, dP; legendre(N + 1, xj, P, dP);
        double dx = -P / dP; xj += dx;
        if (std::fabs(dx) <= 1e-16 * std::max(1.0, std::fabs(xj))) break;
      }
      double P, dP; legendre(N + 1, xj, P, dP);
      B.x[j] = xj; B.w[j] = 2.0 / ((1.0 - xj * xj) * dP * dP);
    }
  } else {
    // Endpoints plus the roots of P_N'; weights 2 / (N(N+1) P_N(x)^2).
    B.x[0] = -1.0; B.x[N] = 1.0;
    for (int j = 1; j < N; ++j) {
      double xj = -std::cos(pi * (j + 0.25) / N - 3.0 / (8.0 * N * pi * (j + 0.25)));
      for (int it = 0; it < 100; ++it) {
        double P, dP; legendre(N, xj, P, dP);
        double d2P = (2.0 * xj * dP - N * (N + 1.0) * P) / (1.0 - xj * xj);
        double dx = -dP / d2P; xj += dx;
        if (std::fabs(dx) <= 1e-16 * std::max(1.0, std::fabs(xj))) break;
      }
      B.x[j] = xj;
    }
    for (int j = 0; j < n; ++j) {
      double P, dP; legendre(N, B.x[j], P, dP);
      B.w[j] = 2.0 / (N * (N + 1.0) * P * P);
    }
  }
  // Enforce the exact mirror symmetry of the node set.
  for (int j = 0; j < n / 2; ++j) {
    double a = 0.5 * (B.x[N - j] - B.x[j]);
    B.x[j] = -a; B.x[N - j] = a;
    double ww = 0.5 * (B.w[j] + B.w[N - j]);
    B.w[j] = ww; B.w[N - j] = ww;
  }
  if (n % 2 == 1) B.x[N / 2] = 0.0;
  // Barycentric weights and the differentiation matrix.
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (B.x[j] - B.x[k]);
  B.D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double dij = (lam[j] / lam[i]) / (B.x[i] - B.x[j]);
      B.D[i * n + j] = dij; s += dij;
    }
    B.D[i * n + i] = -s;
  }
  // Lagrange polynomials at the interval ends, by the product formula.
  B.Lm.assign(n, 1.0); B.Lp.assign(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) {
      if (k == j) continue;
      B.Lm[j] *= (-1.0 - B.x[k]) / (B.x[j] - B.x[k]);
      B.Lp[j] *= (1.0 - B.x[k]) / (B.x[j] - B.x[k]);
    }
  // Split-form operator DS = M^-1 (Q - Q^T), Q = M D, written with the SBP
  // property Q + Q^T = Lp Lp^T - Lm Lm^T as 2 D - M^-1 (Lp Lp^T - Lm Lm^T)
  // (on LGL nodes Lm = e_0, Lp = e_N exactly).
  B.DS.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      B.DS[i * n + j] = 2.0 * B.D[i * n + j] - (B.Lp[i] * B.Lp[j] - B.Lm[i] * B.Lm[j]) / B.w[i];
  return true;
}

// Lagrange basis of an arbitrary node set evaluated at a point.
static double lagrange(const std::vector<double>& xs, int j, double xi) {
  double v = 1.0;
  for (size_t k = 0; k < xs.size(); ++k)
    if ((int)k != j) v *= (xi - xs[k]) / (xs[j] - xs[k]);
  return v;
}

// ---------------------------------------------------------------------------
// Configuration and mesh.
// ---------------------------------------------------------------------------
struct Config {
  int N = 3, nodes = 0, form = 0, physics = 0;
  int twopoint = 0;     // 0 = Chandrashekar, 1 = central average (test switch)
  int dissipation = 1;  // 1 = Rusanov, 0 = none (test switch), 2 = Roe with the Harten-Hyman entropy fix
  int mms = 0;          // 1 = add the manufactured-solution source
  int integrator = 0;   // 0 = LSERK4(5) (Carpenter & Kennedy), 1 = LSERK4-14 (Niegemann, Diehl & Busch)
  int viscosity = 0;    // 0 = constant mu, 1 = Sutherland's law mu(T)
  int hybrid = 0;       // split form: 1 = hybridised/entropy-projection form also on LGL nodes (test switch)
  int fv = 0;           // 1 = FV sub-cell elements enabled (Euler; per-element mask)
  double gamma = 1.4, mu = 0.0, Pr = 0.72, R = 1.0;
  double Tref = 1.0, Ts = 110.4 / 273.15;   // Sutherland: reference temperature, S / Tref
  double mms_A = 0.1, mms_a = 1.0;
};

// Face-local index convention.  Local face f of a hexahedron: f/2 is the
// reference direction of its normal, f%2 = 0 is the "-1" end and 1 the "+1"
// end.  Face-local indices (p,q) are the two tangential volume indices in
// increasing direction order; l runs along the normal line.
static inline void vol_ijk(int f, int p, int q, int l, int& i, int& j, int& k) {
  switch (f / 2) {
    case 0: i = l; j = p; k = q; break;
    case 1: i = p; j = l; k = q; break;
    default: i = p; j = q; k = l; break;
  }
}
// Orientation code o maps the master's (p,q) to the slave's (p',q'):
// swap if bit 2, then reverse the first index if bit 0, the second if bit 1.
static inline void orient_fwd(int o, int N, int p, int q, int& pp, int& qq) {
  int a = (o & 4) ? q : p, b = (o & 4) ? p : q;
  if (o & 1) a = N - a;
  if (o & 2) b = N - b;
  pp = a; qq = b;
}
static inline void orient_inv(int o, int N, int pp, int qq, int& p, int& q) {
  int a = pp, b = qq;
  if (o & 1) a = N - a;
  if (o & 2) b = N - b;
  if (o & 4) { p = b; q = a; } else { p = a; q = b; }
}

// Carpenter & Kennedy (1994) five-stage, fourth-order 2N-storage scheme.
static void lserk_coeffs(double* A, double* B, double* C) {
  const double a[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                       -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
  const double b[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                       1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                       2277821191437.0 / 14882151754819.0};
  const double c[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                       2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};
  for (int s = 0; s < 5; ++s) { A[s] = a[s]; B[s] = b[s]; C[s] = c[s]; }
}

// Niegemann, Diehl & Busch (2012) fourteen-stage, fourth-order 2N-storage
// scheme with a stability region fitted to DG spectra (their RK4-14 table).
static void lserk14_coeffs(double* A, double* B, double* C) {
  const double a[14] = {0.0, -0.7188012108672410, -0.7785331173421570, -0.0053282796654044,
                        -0.8552979934029281, -3.9564138245774565, -1.5780575380587385, -2.0837094552574054,
                        -0.7483334182761610, -0.7032861106563359, 0.0013917096117681, -0.0932075369637460,
                        -0.9514200470875948, -7.1151571693922548};
  const double b[14] = {0.0367762454319673, 0.3136296607553959, 0.1531848691869027, 0.0030097086818182,
                        0.3326293790646110, 0.2440251405350864, 0.3718879239592277, 0.6204126221582444,
                        0.1524043173028741, 0.0760894927419266, 0.0077604214040978, 0.0024647284755382,
                        0.0780348340049386, 5.5059777270269628};
  const double c[14] = {0.0, 0.0367762454319673, 0.1249685262725025, 0.2446177702277698,
                        0.2476149531070420, 0.2969311120382472, 0.3978149645802642, 0.5270854589440328,
                        0.6981269994175695, 0.8190890835352128, 0.8527059887098624, 0.8604711817462826,
                        0.8627060376969976, 0.8734213127600976};
  for (int s = 0; s < 14; ++s) { A[s] = a[s]; B[s] = b[s]; C[s] = c[s]; }
}

// Coefficients of the chosen scheme; returns its number of stages (0 if unknown).
static int rk_coeffs(int integrator, double* A, double* B, double* C) {
  if (integrator == 0) { lserk_coeffs(A, B, C); return 5; }
  if (integrator == 1) { lserk14_coeffs(A, B, C); return 14; }
  return 0;
}

struct Solver {
  Config C;
  Basis B;
  int n1 = 0, n2 = 0, n3 = 0;
  int nElems = 0, Ngeo = 0, nSides = 0;
  std::vector<double> Xgeo;                  // [3][nElems][Ngeo+1]^3
  std::vector<int> sideElem, sideLoc, sideOrient;
  std::vector<int> elemSide, elemSlot;       // [nElems*6]
  std::vector<double> Vgeo;                  // [n1][Ngeo+1] equispaced -> solution nodes
  // lazily computed geometry
  std::vector<std::vector<double>> Ja;       // per element: [9][n3], index 3*r+n
  std::vector<std::vector<double>> Jdet;     // per element: [n3]
  std::vector<std::vector<double>> Xnode;    // per element: [3][n3]
  std::vector<std::vector<double>> nvec;     // per side: [3][n2] master outward n*s
  // FV sub-cells: (N+1)^3 equidistant sub-cells of the reference element
  std::vector<double> Bsub, Bsubinv;         // Bsub[k*n1+i] = integral of l_i over sub-interval k; inverse
  std::vector<double> Vleginv;               // inverse of Vleg[i*n1+m] = orthonormal Legendre m at node i
  std::vector<int> fvmask;                   // per element: 1 = FV sub-cells
  std::vector<std::vector<double>> Vsub;     // per element: [n3] sub-cell volumes
  std::vector<std::vector<double>> Sint;     // per element: [3 r][3 c][N planes][n2] interior sub-face vectors (+xi_r)
  std::vector<std::vector<double>> Sbnd;     // per side: [3 c][n2] master-outward sub-face vectors
  std::string err;
  double lsA[14], lsB[14], lsC[14];
  int nstages = 5;

  int node(int i, int j, int k) const { return (k * n1 + j) * n1 + i; }
  size_t uidx(int v, int e, int nd) const { return ((size_t)v * nElems + e) * n3 + nd; }
  // Where the residual of (v, e, node) is written: the full-size layout, or,
  // while outpos is set (a sampled evaluation), a compact [5][outn][n3] array
  // with element e at position outpos[e].
  std::vector<int> outpos;
  int outn = 0;
  size_t oidx(int v, int e, int nd) const {
    return outpos.empty() ? uidx(v, e, nd) : ((size_t)v * outn + outpos[e]) * n3 + nd;
  }

  bool setup() {
    nstages = rk_coeffs(C.integrator, lsA, lsB, lsC);
    if (nstages == 0) { err = "unknown integrator"; return false; }
    if (!make_basis(C.N, C.nodes, B)) { err = "bad basis"; return false; }
    if (C.form != 0 && C.form != 1) { err = "unknown volume form"; return false; }
    n1 = C.N + 1; n2 = n1 * n1; n3 = n2 * n1;
    std::vector<double> xg(Ngeo + 1);
    for (int m = 0; m <= Ngeo; ++m) xg[m] = -1.0 + 2.0 * m / Ngeo;
    Vgeo.assign((size_t)n1 * (Ngeo + 1), 0.0);
    for (int i = 0; i < n1; ++i)
      for (int m = 0; m <= Ngeo; ++m) Vgeo[i * (Ngeo + 1) + m] = lagrange(xg, m, B.x[i]);
    elemSide.assign((size_t)nElems * 6, -1); elemSlot.assign((size_t)nElems * 6, -1);
    for (int s = 0; s < nSides; ++s)
      for (int m = 0; m < 2; ++m) {
        int e = sideElem[2 * s + m], f = sideLoc[2 * s + m];
        if (e < 0 || e >= nElems || f < 0 || f > 5 || elemSide[e * 6 + f] != -1) { err = "bad connectivity"; return false; }
        elemSide[e * 6 + f] = s; elemSlot[e * 6 + f] = m;
      }
    for (size_t t = 0; t < elemSide.size(); ++t)
      if (elemSide[t] < 0) { err = "open face"; return false; }
    Ja.assign(nElems, {}); Jdet.assign(nElems, {}); Xnode.assign(nElems, {}); nvec.assign(nSides, {});
    if (C.fv) {
      setup_fv_basis();
      fvmask.assign(nElems, 0);
      Vsub.assign(nElems, {}); Sint.assign(nElems, {}); Sbnd.assign(nSides, {});
    }
    return true;
  }

  // Geometry of element e at the solution nodes (tensor-product interpolation
  // of the equispaced geometry nodes, one direction at a time).
  void ensure_geom(int e) {
    if (!Jdet[e].empty()) return;
    const int g1 = Ngeo + 1;
    std::vector<double>& X = Xnode[e];
    X.assign(3 * (size_t)n3, 0.0);
    // Geometry is interpolated relative to the element's first geometry node
    // x0 (all metric terms are invariant under translation); this keeps the
    // rounding error of the metrics proportional to the element size.
    double x0[3];
    for (int d = 0; d < 3; ++d) {
      const double* xg = &Xgeo[((size_t)d * nElems + e) * g1 * g1 * g1];
      x0[d] = xg[0];
      std::vector<double> t1((size_t)g1 * g1 * n1), t2((size_t)g1 * n1 * n1);
      for (int c = 0; c < g1; ++c)
        for (int b = 0; b < g1; ++b)
          for (int i = 0; i < n1; ++i) {
            double s = 0.0;
            for (int a = 0; a < g1; ++a) s += Vgeo[i * g1 + a] * (xg[(c * g1 + b) * g1 + a] - x0[d]);
            t1[(c * g1 + b) * n1 + i] = s;
          }
      for (int c = 0; c < g1; ++c)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            double s = 0.0;
            for (int b = 0; b < g1; ++b) s += Vgeo[j * g1 + b] * t1[(c * g1 + b) * n1 + i];
            t2[(c * n1 + j) * n1 + i] = s;
          }
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            double s = 0.0;
            for (int c = 0; c < g1; ++c) s += Vgeo[k * g1 + c] * t2[(c * n1 + j) * n1 + i];
            X[(size_t)d * n3 + node(i, j, k)] = s;
          }
    }
    // d/dxi_r of a nodal field along reference direction r.
    auto deriv = [&](const double* f, int r, double* out) {
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            int a = (r == 0) ? i : (r == 1) ? j : k;
            double s = 0.0;
            for (int l = 0; l < n1; ++l) {
              int ii = i, jj = j, kk = k;
              if (r == 0) ii = l; else if (r == 1) jj = l; else kk = l;
              s += B.D[a * n1 + l] * f[node(ii, jj, kk)];
            }
            out[node(i, j, k)] = s;
          }
    };
    std::vector<double> dX(9 * (size_t)n3);  // dX[3*d+r] = dX_d/dxi_r
    for (int d = 0; d < 3; ++d)
      for (int r = 0; r < 3; ++r) deriv(&X[(size_t)d * n3], r, &dX[(size_t)(3 * d + r) * n3]);
    std::vector<double>& J = Jdet[e];
    J.assign(n3, 0.0);
    for (int t = 0; t < n3; ++t) {
      double a[3][3];
      for (int d = 0; d < 3; ++d)
        for (int r = 0; r < 3; ++r) a[d][r] = dX[(size_t)(3 * d + r) * n3 + t];
      J[t] = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
             a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
    }
    // Conservative curl form (Kopriva 2006): Ja^r_n = -[curl_xi (X_l grad_xi X_m)]_r,
    // (n,m,l) cyclic, with the product collocated at the solution nodes.
    std::vector<double>& M = Ja[e];
    M.assign(9 * (size_t)n3, 0.0);
    std::vector<double> V(3 * (size_t)n3);
    for (int nn = 0; nn < 3; ++nn) {
      int m = (nn + 1) % 3, l = (nn + 2) % 3;
      for (int s = 0; s < 3; ++s)
        for (int t = 0; t < n3; ++t)
          V[(size_t)s * n3 + t] = X[(size_t)l * n3 + t] * dX[(size_t)(3 * m + s) * n3 + t];
      // curl components: c_0 = d1 V2 - d2 V1, c_1 = d2 V0 - d0 V2, c_2 = d0 V1 - d1 V0
      std::vector<double> a(n3), b(n3);
      for (int r = 0; r < 3; ++r) {
        int r1 = (r + 1) % 3, r2 = (r + 2) % 3;
        deriv(&V[(size_t)r2 * n3], r1, a.data());
        deriv(&V[(size_t)r1 * n3], r2, b.data());
        for (int t = 0; t < n3; ++t) M[(size_t)(3 * r + nn) * n3 + t] = -(a[t] - b[t]);
      }
    }
    for (int d = 0; d < 3; ++d)
      for (int t = 0; t < n3; ++t) X[(size_t)d * n3 + t] += x0[d];
  }

  void ensure_side(int s) {
    if (!nvec[s].empty()) return;
    int e = sideElem[2 * s], f = sideLoc[2 * s];
    ensure_geom(e);
    const int d = f / 2;
    const double sg = (f % 2) ? 1.0 : -1.0;
    const std::vector<double>& L = (f % 2) ? B.Lp : B.Lm;
    nvec[s].assign(3 * (size_t)n2, 0.0);
    for (int q = 0; q < n1; ++q)
      for (int p = 0; p < n1; ++p)
        for (int c = 0; c < 3; ++c) {
          double v = 0.0;
          for (int l = 0; l < n1; ++l) {
            int i, j, k; vol_ijk(f, p, q, l, i, j, k);
            v += L[l] * Ja[e][(size_t)(3 * d + c) * n3 + node(i, j, k)];
          }
          nvec[s][(size_t)c * n2 + q * n1 + p] = sg * v;
        }
  }

  bool check_jacobians() {
    for (int e = 0; e < nElems; ++e) {
      ensure_geom(e);
      for (int t = 0; t < n3; ++t)
        if (!(Jdet[e][t] > 0.0)) { err = "non-positive Jacobian"; return false; }
    }
    return true;
  }

  // -------------------------------------------------------------------------
  // Physics (paper eq. for F; perfect gas).
  // -------------------------------------------------------------------------
  template <class T> void prim(const T* U, T& rho, T* u, T& p) const {
    rho = U[0];
    for (int d = 0; d < 3; ++d) u[d] = U[1 + d] / rho;
    p = (C.gamma - 1.0) * (U[4] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
  }
  // Advective flux in the (not necessarily unit) direction nv.
  template <class T> void flux_adv(const T* U, const double* nv, T* F) const {
    T rho, u[3], p; prim(U, rho, u, p);
    T un = u[0] * nv[0] + u[1] * nv[1] + u[2] * nv[2];
    F[0] = rho * un;
    for (int d = 0; d < 3; ++d) F[1 + d] = U[1 + d] * un + p * nv[d];
    F[4] = (U[4] + p) * un;
  }
  // Logarithmic mean (x - y) / (ln x - ln y), with the atanh series near x = y.
  template <class T> T logmean(const T& x, const T& y) const {
    T f = (x - y) / (x + y);
    T u = f * f;
    if (val(u) < 1e-4)
      return (x + y) / (2.0 + u * (2.0 / 3.0 + u * (2.0 / 5.0 + u * (2.0 / 7.0))));
    return (x - y) / (log(x) - log(y));
  }
  // Two-point volume flux in direction nv (linear in nv).
  template <class T> void flux_twopoint(const T* Ua, const T* Ub, const double* nv, T* F) const {
    if (C.twopoint == 1) {
      T Fa[5], Fb[5];
      flux_adv(Ua, nv, Fa); flux_adv(Ub, nv, Fb);
      for (int v = 0; v < 5; ++v) F[v] = 0.5 * (Fa[v] + Fb[v]);
      return;
    }
    // Chandrashekar (2013): beta = rho/(2p); rho^ln, beta^ln logarithmic
    // means; p_hat = {rho}/(2{beta}).
    T ra, ua[3], pa, rb, ub[3], pb;
    prim(Ua, ra, ua, pa); prim(Ub, rb, ub, pb);
    T ba = ra / (2.0 * pa), bb = rb / (2.0 * pb);
    T rho_ln = logmean(ra, rb), beta_ln = logmean(ba, bb);
    T um[3];
    for (int d = 0; d < 3; ++d) um[d] = 0.5 * (ua[d] + ub[d]);
    T phat = 0.5 * (ra + rb) / (2.0 * (0.5 * (ba + bb)));
    T u2m = 0.5 * ((ua[0] * ua[0] + ua[1] * ua[1] + ua[2] * ua[2]) + (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]));
    T umn = um[0] * nv[0] + um[1] * nv[1] + um[2] * nv[2];
    F[0] = rho_ln * umn;
    for (int d = 0; d < 3; ++d) F[1 + d] = phat * nv[d] + um[d] * F[0];
    F[4] = F[0] * (1.0 / (2.0 * (C.gamma - 1.0) * beta_ln) - 0.5 * u2m) +
           (um[0] * F[1] + um[1] * F[2] + um[2] * F[3]);
  }
  // Dynamic viscosity at temperature temp: constant, or Sutherland's law
  // mu = mu_ref (T/Tref)^(3/2) (1 + S/Tref) / (T/Tref + S/Tref) with mu_ref = C.mu
  // the viscosity at Tref (the TGV section's temperature-dependent viscosity).
  template <class T> T viscosity(const T& temp) const {
    if (C.viscosity == 0) return T(C.mu);
    const T th = temp / C.Tref;
    return C.mu * th * sqrt(th) * (1.0 + C.Ts) / (th + C.Ts);
  }
  // Viscous flux G_n(U, grad) in Cartesian direction n; grad[3*a+d] = dq_a/dx_d,
  // q = (u, v, w, T).  Newtonian stress with Stokes' hypothesis, Fourier heat
  // flux with the conductivity of constant Prandtl number.
  template <class T> void flux_visc(const T* U, const T* g, int n, T* G) const {
    T rho, u[3], p; prim(U, rho, u, p);
    const T mu = viscosity(T(p / (rho * C.R)));
    const T lam = mu * (C.gamma * C.R / ((C.gamma - 1.0) * C.Pr));
    T divu = g[0] + g[4] + g[8];
    T tau[3];
    for (int a = 0; a < 3; ++a) {
      tau[a] = mu * (g[3 * a + n] + g[3 * n + a]);
      if (a == n) tau[a] = tau[a] - (2.0 / 3.0) * mu * divu;
    }
    G[0] = T(0.0);
    for (int a = 0; a < 3; ++a) G[1 + a] = tau[a];
    G[4] = tau[0] * u[0] + tau[1] * u[1] + tau[2] * u[2] + lam * g[9 + n];
  }

  // Roe's linearisation (Roe 1981) across a face with unit normal nh: Roe
  // averages, the five waves (two acoustic, entropy, two shear) and their
  // strengths.  mode 0: D = |A~|(UR-UL), with the Harten & Hyman (1983)
  // entropy fix on the acoustic speeds (delta = max(0, l~ - l(UL), l(UR) - l~);
  // |l~| < delta becomes (l~^2 + delta^2)/(2 delta)); mode 1: A~(UR-UL) with
  // signed speeds (Roe's property: equals f(UR).nh - f(UL).nh); mode 2: |A~|(UR-UL)
  // without the fix.
  template <class T> void roe_matrix(const T* UL, const T* UR, const double* nh, int mode, T* D) const {
    T rl, ul[3], pl, rr, ur[3], pr;
    prim(UL, rl, ul, pl); prim(UR, rr, ur, pr);
    const T HL = (UL[4] + pl) / rl, HR = (UR[4] + pr) / rr;
    const T sl = sqrt(rl), sr = sqrt(rr), ws = sl + sr;
    T um[3];
    for (int d = 0; d < 3; ++d) um[d] = (sl * ul[d] + sr * ur[d]) / ws;
    const T Hm = (sl * HL + sr * HR) / ws;
    const T q2 = um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
    const T c2 = (C.gamma - 1.0) * (Hm - 0.5 * q2);
    const T cm = sqrt(c2);
    const T rm = sl * sr;
    const T unm = um[0] * nh[0] + um[1] * nh[1] + um[2] * nh[2];
    const T dr = rr - rl, dp = pr - pl;
    T du[3];
    for (int d = 0; d < 3; ++d) du[d] = ur[d] - ul[d];
    const T dun = du[0] * nh[0] + du[1] * nh[1] + du[2] * nh[2];
    const T a1 = (dp - rm * cm * dun) / (2.0 * c2);
    const T a5 = (dp + rm * cm * dun) / (2.0 * c2);
    const T a2 = dr - dp / c2;
    T l1 = unm - cm, l2 = unm, l5 = unm + cm;
    if (mode != 1) {
      l2 = absv(l2);
      T fix[2] = {l1, l5};
      const T cl = sqrt(C.gamma * pl / rl), cr = sqrt(C.gamma * pr / rr);
      const T unl = ul[0] * nh[0] + ul[1] * nh[1] + ul[2] * nh[2];
      const T unr = ur[0] * nh[0] + ur[1] * nh[1] + ur[2] * nh[2];
      const T lL[2] = {unl - cl, unl + cl}, lR[2] = {unr - cr, unr + cr};
      for (int k = 0; k < 2; ++k) {
        T a = absv(fix[k]);
        if (mode == 0) {
          const T delta = maxv(maxv(T(0.0), T(fix[k] - lL[k])), T(lR[k] - fix[k]));
          if (val(a) < val(delta)) a = (fix[k] * fix[k] + delta * delta) / (2.0 * delta);
        }
        fix[k] = a;
      }
      l1 = fix[0]; l5 = fix[1];
    }
    // acoustic waves r1,5 = (1, u~ -+ c~ n, H~ -+ un~ c~), entropy wave (1, u~, q2/2),
    // shear waves rho~ (0, du - dun n, u~.du - un~ dun)
    const T udu = um[0] * du[0] + um[1] * du[1] + um[2] * du[2];
    D[0] = l1 * a1 + l2 * a2 + l5 * a5;
    for (int d = 0; d < 3; ++d)
      D[1 + d] = l1 * a1 * (um[d] - cm * nh[d]) + l2 * (a2 * um[d] + rm * (du[d] - dun * nh[d])) +
                 l5 * a5 * (um[d] + cm * nh[d]);
    D[4] = l1 * a1 * (Hm - unm * cm) + l2 * (a2 * 0.5 * q2 + rm * (udu - unm * dun)) + l5 * a5 * (Hm + unm * cm);
  }

  // Entropy variables of the mathematical entropy S = -rho s/(gamma-1),
  // s = ln p - gamma ln rho (the entropy the Chandrashekar flux conserves):
  // v = dS/dU = ((gamma - s)/(gamma-1) - rho|u|^2/(2p), rho u/p, -rho/p).
  template <class T> void entropy_vars(const T* U, T* v) const {
    T rho, u[3], p; prim(U, rho, u, p);
    const T s = log(p) - C.gamma * log(rho);
    const T b = rho / p;
    v[0] = (C.gamma - s) / (C.gamma - 1.0) - 0.5 * b * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int d = 0; d < 3; ++d) v[1 + d] = b * u[d];
    v[4] = -b;
  }
  // Inverse of entropy_vars: with b = rho/p = -v_4 the velocity is v_{1..3}/b,
  // s follows from v_0, and s = ln p - gamma ln rho with p = rho/b gives
  // ln rho = -(s + ln b)/(gamma - 1).
  template <class T> void cons_from_entropy(const T* v, T* U) const {
    const T b = -v[4];
    T u[3];
    for (int d = 0; d < 3; ++d) u[d] = v[1 + d] / b;
    const T q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T s = C.gamma - (C.gamma - 1.0) * (v[0] + 0.5 * b * q2);
    const T rho = exp(-(s + log(b)) / (C.gamma - 1.0));
    const T p = rho / b;
    U[0] = rho;
    for (int d = 0; d < 3; ++d) U[1 + d] = rho * u[d];
    U[4] = p / (C.gamma - 1.0) + 0.5 * rho * q2;
  }
  // Split form through the hybridised operator with entropy projection:
  // always on LG nodes, on LGL nodes only when asked for (there it reduces
  // to the plain split form).
  bool hybrid() const { return C.form == 1 && (C.nodes == 0 || C.hybrid == 1); }

  // Manufactured solution of the convergence section:
  // rho = 2 + A sin(2 pi (x+y+z - a t)), rho u = rho, rho e = rho^2.
  void mms_source(double x, double y, double z, double t, double* Q) const {
    const double pi = std::acos(-1.0), A = C.mms_A, a = C.mms_a, g = C.gamma;
    double ph = 2.0 * pi * (x + y + z - a * t);
    double r = 2.0 + A * std::sin(ph);
    double r1 = 2.0 * pi * A * std::cos(ph);
    double r2 = -4.0 * pi * pi * A * std::sin(ph);
    Q[0] = (3.0 - a) * r1;
    double qm = (3.0 - a) * r1 + (g - 1.0) * (2.0 * r - 1.5) * r1;
    Q[1] = qm; Q[2] = qm; Q[3] = qm;
    Q[4] = (6.0 - 2.0 * a) * r * r1 + 3.0 * (g - 1.0) * (2.0 * r - 1.5) * r1 - 3.0 * C.mu * g * r2 / C.Pr;
  }

  // -------------------------------------------------------------------------
  // The residual.  U, Ut: [5][nElems][n3].  If elist is non-empty only those
  // elements of Ut are written (and only the data they need is computed).
  // -------------------------------------------------------------------------
  template <class T> struct Work {
    std::vector<std::vector<T>> tr;     // per side: [2][5][n2] U traces (master indexing)
    std::vector<std::vector<T>> g;      // per element: [12][n3] lifted gradients
    std::vector<std::vector<T>> gtr;    // per side: [2][12][n2] gradient traces
    // FV sub-cells: per element the sub-cell means [5][n3], and (Navier-Stokes)
    // the sub-cell gradients [12][n3]: Green-Gauss for FV elements, the
    // sub-cell means of the lifted gradient for DG elements
    std::vector<std::vector<T>> fvc, fvg;
  };

  // Face traces of both sides.  Plain interpolation of U, or, in the
  // hybridised split form, the entropy-projected state u(E v(U)): the
  // entropy variables are interpolated and mapped back.
  template <class T> void side_traces(const T* U, int s, Work<T>& W) {
    if (!W.tr[s].empty()) return;
    W.tr[s].assign(2 * 5 * (size_t)n2, T(0.0));
    for (int m = 0; m < 2; ++m) {
      int e = sideElem[2 * s + m], f = sideLoc[2 * s + m];
      const std::vector<double>& L = (f % 2) ? B.Lp : B.Lm;
      for (int q = 0; q < n1; ++q)
        for (int p = 0; p < n1; ++p) {
          int pp = p, qq = q;
          if (m == 1) orient_fwd(sideOrient[s], C.N, p, q, pp, qq);
          T acc[5];
          for (int v = 0; v < 5; ++v) acc[v] = T(0.0);
          for (int l = 0; l < n1; ++l) {
            int i, j, k; vol_ijk(f, pp, qq, l, i, j, k);
            T Ul[5], x[5];
            for (int v = 0; v < 5; ++v) Ul[v] = U[uidx(v, e, node(i, j, k))];
            if (hybrid()) entropy_vars(Ul, x);
            else for (int v = 0; v < 5; ++v) x[v] = Ul[v];
            for (int v = 0; v < 5; ++v) acc[v] += L[l] * x[v];
          }
          T tr[5];
          if (hybrid()) cons_from_entropy(acc, tr);
          else for (int v = 0; v < 5; ++v) tr[v] = acc[v];
          for (int v = 0; v < 5; ++v) W.tr[s][((size_t)m * 5 + v) * n2 + q * n1 + p] = tr[v];
        }
    }
  }

  template <class T> void lift_elem(const T* U, int e, Work<T>& W) {
    if (!W.g[e].empty()) return;
    ensure_geom(e);
    for (int f = 0; f < 6; ++f) { side_traces(U, elemSide[e * 6 + f], W); ensure_side(elemSide[e * 6 + f]); }
    if (C.fv) ensure_fv_caches(W);
    std::vector<T> q(4 * (size_t)n3);
    for (int t = 0; t < n3; ++t) {
      T Ul[5]; for (int v = 0; v < 5; ++v) Ul[v] = U[uidx(v, e, t)];
      T rho, u[3], p; prim(Ul, rho, u, p);
      q[t] = u[0]; q[n3 + t] = u[1]; q[2 * (size_t)n3 + t] = u[2]; q[3 * (size_t)n3 + t] = p / (rho * C.R);
    }
    std::vector<T>& g = W.g[e];
    g.assign(12 * (size_t)n3, T(0.0));
    const std::vector<double>& M = Ja[e];
    // Volume part of eq. (dgsem_lifted): -sum_r sum_l (w_l/w_a) D_{l a} (Ja^r_d q)_l.
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          int t = node(i, j, k);
          for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 3; ++d) {
              T acc(0.0);
              for (int r = 0; r < 3; ++r) {
                int ai = (r == 0) ? i : (r == 1) ? j : k;
                for (int l = 0; l < n1; ++l) {
                  int ii = i, jj = j, kk = k;
                  if (r == 0) ii = l; else if (r == 1) jj = l; else kk = l;
                  int tl = node(ii, jj, kk);
                  double c = B.w[l] / B.w[ai] * B.D[l * n1 + ai];
                  acc -= c * (M[(size_t)(3 * r + d) * n3 + tl] * q[(size_t)a * n3 + tl]);
                }
              }
              g[(size_t)(3 * a + d) * n3 + t] = acc;
            }
        }
    // Surface part: (1/w) l(+-1) {q} (n s)_d with the outward normal.
    for (int f = 0; f < 6; ++f) {
      int s = elemSide[e * 6 + f], m = elemSlot[e * 6 + f];
      const std::vector<double>& L = (f % 2) ? B.Lp : B.Lm;
      for (int qq = 0; qq < n1; ++qq)
        for (int pp = 0; pp < n1; ++pp) {
          int p = pp, q2 = qq;
          if (m == 1) orient_inv(sideOrient[s], C.N, pp, qq, p, q2);
          int fi = q2 * n1 + p;
          T qa[4], qb[4];
          for (int side = 0; side < 2; ++side) {
            T Ul[5]; for (int v = 0; v < 5; ++v) Ul[v] = W.tr[s][((size_t)side * 5 + v) * n2 + fi];
            T rho, u[3], pr; prim(Ul, rho, u, pr);
            T* qx = side == 0 ? qa : qb;
            qx[0] = u[0]; qx[1] = u[1]; qx[2] = u[2]; qx[3] = pr / (rho * C.R);
          }
          if (C.fv && side_fv(s)) {
            // the other side is an FV element: its q at this face node is the
            // face polynomial whose sub-face means are its layer-0 values
            T qf[4];
            fv_face_q(U, e, f, pp, qq, W, qf);
            T* qo = (m == 0) ? qb : qa;
            for (int a = 0; a < 4; ++a) qo[a] = qf[a];
          }
          double ns[3];
          for (int c = 0; c < 3; ++c) ns[c] = (m == 0 ? 1.0 : -1.0) * nvec[s][(size_t)c * n2 + fi];
          for (int l = 0; l < n1; ++l) {
            int i, j, k; vol_ijk(f, pp, qq, l, i, j, k);
            int t = node(i, j, k);
            double c = L[l] / B.w[l];
            for (int a = 0; a < 4; ++a) {
              T avg = 0.5 * (qa[a] + qb[a]);
              for (int d = 0; d < 3; ++d) g[(size_t)(3 * a + d) * n3 + t] += c * (avg * ns[d]);
            }
          }
        }
    }
    for (size_t c = 0; c < 12; ++c)
      for (int t = 0; t < n3; ++t) g[c * n3 + t] = g[c * n3 + t] / Jdet[e][t];
  }

  template <class T> void side_grad_traces(const T* U, int s, Work<T>& W) {
    if (!W.gtr[s].empty()) return;
    W.gtr[s].assign(2 * 12 * (size_t)n2, T(0.0));
    for (int m = 0; m < 2; ++m) {
      int e = sideElem[2 * s + m], f = sideLoc[2 * s + m];
      lift_elem(U, e, W);
      const std::vector<double>& L = (f % 2) ? B.Lp : B.Lm;
      for (int q = 0; q < n1; ++q)
        for (int p = 0; p < n1; ++p) {
          int pp = p, qq = q;
          if (m == 1) orient_fwd(sideOrient[s], C.N, p, q, pp, qq);
          for (int c = 0; c < 12; ++c) {
            T acc(0.0);
            for (int l = 0; l < n1; ++l) {
              int i, j, k; vol_ijk(f, pp, qq, l, i, j, k);
              acc += L[l] * W.g[e][(size_t)c * n3 + node(i, j, k)];
            }
            W.gtr[s][((size_t)m * 12 + c) * n2 + q * n1 + p] = acc;
          }
        }
    }
  }

  // Outward (master) surface flux Phi at every face node of side s: [5][n2].
  template <class T> void side_flux(const T* U, int s, Work<T>& W, std::vector<T>& Phi) {
    side_traces(U, s, W);
    ensure_side(s);
    if (C.physics == 1) side_grad_traces(U, s, W);
    Phi.assign(5 * (size_t)n2, T(0.0));
    for (int fi = 0; fi < n2; ++fi) {
      T UL[5], UR[5];
      for (int v = 0; v < 5; ++v) {
        UL[v] = W.tr[s][(size_t)v * n2 + fi];
        UR[v] = W.tr[s][((size_t)5 + v) * n2 + fi];
      }
      double nv[3], nh[3];
      for (int c = 0; c < 3; ++c) nv[c] = nvec[s][(size_t)c * n2 + fi];
      double sA = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      for (int c = 0; c < 3; ++c) nh[c] = nv[c] / sA;
      T Fc[5];
      if (C.form == 1) {
        flux_twopoint(UL, UR, nv, Fc);
      } else {
        T FL[5], FR[5];
        flux_adv(UL, nv, FL); flux_adv(UR, nv, FR);
        for (int v = 0; v < 5; ++v) Fc[v] = 0.5 * (FL[v] + FR[v]);
      }
      if (C.dissipation == 2) {
        // Roe: central part minus (1/2)|A~|(UR - UL), on the unit normal, times s
        T D[5];
        roe_matrix(UL, UR, nh, 0, D);
        for (int v = 0; v < 5; ++v) Phi[(size_t)v * n2 + fi] = Fc[v] - 0.5 * sA * D[v];
      } else {
        T lmax(0.0);
        if (C.dissipation) {
          T rl, ul[3], pl, rr, ur[3], pr;
          prim(UL, rl, ul, pl); prim(UR, rr, ur, pr);
          T cl = sqrt(C.gamma * pl / rl), cr = sqrt(C.gamma * pr / rr);
          T unl = ul[0] * nh[0] + ul[1] * nh[1] + ul[2] * nh[2];
          T unr = ur[0] * nh[0] + ur[1] * nh[1] + ur[2] * nh[2];
          lmax = maxv(T(absv(unl) + cl), T(absv(unr) + cr));
        }
        for (int v = 0; v < 5; ++v) Phi[(size_t)v * n2 + fi] = Fc[v] - 0.5 * (lmax * sA) * (UR[v] - UL[v]);
      }
      if (C.physics == 1) {
        T gL[12], gR[12];
        for (int c = 0; c < 12; ++c) {
          gL[c] = W.gtr[s][(size_t)c * n2 + fi];
          gR[c] = W.gtr[s][((size_t)12 + c) * n2 + fi];
        }
        for (int n = 0; n < 3; ++n) {
          T GL[5], GR[5];
          flux_visc(UL, gL, n, GL); flux_visc(UR, gR, n, GR);
          for (int v = 0; v < 5; ++v) Phi[(size_t)v * n2 + fi] -= 0.5 * (GL[v] + GR[v]) * nv[n];
        }
      }
    }
  }

  template <class T> void residual_elem(const T* U, int e, Work<T>& W, std::vector<std::vector<T>>& sflux,
                                        T* Ut, double t) {
    ensure_geom(e);
    const std::vector<double>& M = Ja[e];
    std::vector<T> V(5 * (size_t)n3, T(0.0));
    auto Uat = [&](int tt, T* out) { for (int v = 0; v < 5; ++v) out[v] = U[uidx(v, e, tt)]; };
    // Contravariant fluxes Ftilde^r = sum_n Ja^r_n F_n at every node.
    // (weak form: advective + viscous; split form: viscous only)
    std::vector<T> Ft(15 * (size_t)n3, T(0.0));
    for (int tt = 0; tt < n3; ++tt) {
      T Ul[5]; Uat(tt, Ul);
      for (int r = 0; r < 3; ++r) {
        double nv[3] = {M[(size_t)(3 * r + 0) * n3 + tt], M[(size_t)(3 * r + 1) * n3 + tt], M[(size_t)(3 * r + 2) * n3 + tt]};
        T F[5] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
        if (C.form == 0) flux_adv(Ul, nv, F);
        if (C.physics == 1) {
          T gl[12];
          for (int c = 0; c < 12; ++c) gl[c] = W.g[e][(size_t)c * n3 + tt];
          for (int n = 0; n < 3; ++n) {
            T G[5]; flux_visc(Ul, gl, n, G);
            for (int v = 0; v < 5; ++v) F[v] = F[v] - G[v] * nv[n];
          }
        }
        for (int v = 0; v < 5; ++v) Ft[(size_t)(5 * r + v) * n3 + tt] = F[v];
      }
    }
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          int tt = node(i, j, k);
          for (int r = 0; r < 3; ++r) {
            int a = (r == 0) ? i : (r == 1) ? j : k;
            for (int l = 0; l < n1; ++l) {
              int ii = i, jj = j, kk = k;
              if (r == 0) ii = l; else if (r == 1) jj = l; else kk = l;
              int tl = node(ii, jj, kk);
              // weak-form volume term: sum_l (w_l/w_a) D_{l a} Ftilde^r_l
              double c = B.w[l] / B.w[a] * B.D[l * n1 + a];
              for (int v = 0; v < 5; ++v) V[(size_t)v * n3 + tt] += c * Ft[(size_t)(5 * r + v) * n3 + tl];
              if (C.form == 1 && !hybrid() && l != a) {
                // flux differencing: -sum_l DS_{a l} F#(U_tt, U_tl) . avg(Ja^r)
                T Ua[5], Ub[5]; Uat(tt, Ua); Uat(tl, Ub);
                double nv[3];
                for (int c2 = 0; c2 < 3; ++c2)
                  nv[c2] = 0.5 * (M[(size_t)(3 * r + c2) * n3 + tt] + M[(size_t)(3 * r + c2) * n3 + tl]);
                T F[5]; flux_twopoint(Ua, Ub, nv, F);
                double ds = B.DS[a * n1 + l];
                for (int v = 0; v < 5; ++v) V[(size_t)v * n3 + tt] -= ds * F[v];
              }
            }
          }
        }
    if (hybrid())
      for (int r = 0; r < 3; ++r)
        for (int qq = 0; qq < n1; ++qq)
          for (int pp = 0; pp < n1; ++pp) hybrid_line(U, e, r, pp, qq, V);
    // Surface term: -(1/w) l(+-1) Phi_out for each of the six faces.
    for (int f = 0; f < 6; ++f) {
      int s = elemSide[e * 6 + f], m = elemSlot[e * 6 + f];
      const std::vector<double>& L = (f % 2) ? B.Lp : B.Lm;
      const std::vector<T>& Phi = sflux[s];
      for (int qq = 0; qq < n1; ++qq)
        for (int pp = 0; pp < n1; ++pp) {
          int p = pp, q2 = qq;
          if (m == 1) orient_inv(sideOrient[s], C.N, pp, qq, p, q2);
          int fi = q2 * n1 + p;
          for (int l = 0; l < n1; ++l) {
            int i, j, k; vol_ijk(f, pp, qq, l, i, j, k);
            int tt = node(i, j, k);
            double c = L[l] / B.w[l];
            for (int v = 0; v < 5; ++v) {
              T ph = (m == 0) ? Phi[(size_t)v * n2 + fi] : T(-Phi[(size_t)v * n2 + fi]);
              V[(size_t)v * n3 + tt] -= c * ph;
            }
          }
        }
    }
    for (int v = 0; v < 5; ++v)
      for (int tt = 0; tt < n3; ++tt) Ut[oidx(v, e, tt)] = V[(size_t)v * n3 + tt] / Jdet[e][tt];
    if (C.mms) {
      for (int tt = 0; tt < n3; ++tt) {
        double Q[5];
        mms_source(Xnode[e][tt], Xnode[e][n3 + tt], Xnode[e][2 * (size_t)n3 + tt], t, Q);
        for (int v = 0; v < 5; ++v) Ut[oidx(v, e, tt)] += Q[v];
      }
    }
  }

  // -------------------------------------------------------------------------
  // FV sub-cells (shock capturing; paper: "Governing Equations and Numerical
  // Method", the FV sub-cell scheme of Sonntag & Munz with (N+1)^3 integral
  // means per element).  Reading: equidistant reference sub-cells; DG <-> FV
  // by exact sub-cell integral means of J U; sub-cell volumes and face
  // vectors as exact integrals of the J and Ja^r interpolants; second-order
  // MUSCL reconstruction of primitive variables with the minmod limiter, the
  // neighbour element's first sub-cell layer serving as ghost cell; Rusanov
  // flux on every sub-face; a face with an FV element on either side is
  // evaluated on sub-faces from both sides' first two sub-cell layers (a DG
  // side contributes its sub-cell means), and a DG element takes it back as
  // the face polynomial with those sub-face integrals.
  // -------------------------------------------------------------------------
  static void invert(std::vector<double> A, int n, std::vector<double>& inv) {
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
      int piv = c;
      for (int r = c + 1; r < n; ++r)
        if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
      for (int k = 0; k < n; ++k) { std::swap(A[c * n + k], A[piv * n + k]); std::swap(inv[c * n + k], inv[piv * n + k]); }
      const double d = A[c * n + c];
      for (int k = 0; k < n; ++k) { A[c * n + k] /= d; inv[c * n + k] /= d; }
      for (int r = 0; r < n; ++r) {
        if (r == c) continue;
        const double f = A[r * n + c];
        for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
      }
    }
  }
  // Sub-interval k of [-1,1]: [-1 + 2k/(N+1), -1 + 2(k+1)/(N+1)].
  double sub_edge(int k) const { return -1.0 + 2.0 * k / n1; }
  void setup_fv_basis() {
    Basis G; make_basis(C.N, 0, G);   // Gauss rule, exact for the degree-N integrands
    Bsub.assign((size_t)n1 * n1, 0.0);
    for (int k = 0; k < n1; ++k) {
      const double a = sub_edge(k), b = sub_edge(k + 1);
      for (int i = 0; i < n1; ++i) {
        double s = 0.0;
        for (int g = 0; g < n1; ++g) s += G.w[g] * lagrange(B.x, i, a + 0.5 * (b - a) * (G.x[g] + 1.0));
        Bsub[k * n1 + i] = 0.5 * (b - a) * s;
      }
    }
    invert(Bsub, n1, Bsubinv);
    std::vector<double> V((size_t)n1 * n1);
    for (int i = 0; i < n1; ++i)
      for (int m = 0; m < n1; ++m) {
        double P, dP; legendre(m, B.x[i], P, dP);
        V[i * n1 + m] = std::sqrt((2.0 * m + 1.0) / 2.0) * P;
      }
    invert(V, n1, Vleginv);
  }
  // Tensor-product application of a 1-D operator M (n1 x n1) along all three directions.
  template <class T> void apply3(const std::vector<double>& M, const T* in, T* out) const {
    std::vector<T> a((size_t)n3), b((size_t)n3);
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          T s(0.0);
          for (int l = 0; l < n1; ++l) s += M[i * n1 + l] * in[node(l, j, k)];
          a[node(i, j, k)] = s;
        }
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          T s(0.0);
          for (int l = 0; l < n1; ++l) s += M[j * n1 + l] * a[node(i, l, k)];
          b[node(i, j, k)] = s;
        }
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          T s(0.0);
          for (int l = 0; l < n1; ++l) s += M[k * n1 + l] * b[node(i, j, l)];
          out[node(i, j, k)] = s;
        }
  }
  // Sub-cell volumes and interior sub-face vectors of element e.
  void ensure_fv_geom(int e) {
    if (!Vsub[e].empty()) return;
    ensure_geom(e);
    Vsub[e].assign(n3, 0.0);
    apply3(Bsub, Jdet[e].data(), Vsub[e].data());
    const int N = C.N;
    Sint[e].assign((size_t)9 * N * n2, 0.0);
    for (int r = 0; r < 3; ++r)
      for (int kk = 0; kk < N; ++kk) {
        const double xp = sub_edge(kk + 1);
        std::vector<double> lp(n1);
        for (int l = 0; l < n1; ++l) lp[l] = lagrange(B.x, l, xp);
        for (int c = 0; c < 3; ++c) {
          // Ja^r_c on the plane xi_r = xp at the tangential nodes, then integrated over each sub-face
          std::vector<double> pl(n2, 0.0);
          for (int b2 = 0; b2 < n1; ++b2)
            for (int a2 = 0; a2 < n1; ++a2)
              for (int l = 0; l < n1; ++l) {
                int i, j, k; vol_ijk(2 * r, a2, b2, l, i, j, k);
                pl[b2 * n1 + a2] += lp[l] * Ja[e][(size_t)(3 * r + c) * n3 + node(i, j, k)];
              }
          for (int q = 0; q < n1; ++q)
            for (int p = 0; p < n1; ++p) {
              double s = 0.0;
              for (int b2 = 0; b2 < n1; ++b2)
                for (int a2 = 0; a2 < n1; ++a2) s += Bsub[p * n1 + a2] * Bsub[q * n1 + b2] * pl[b2 * n1 + a2];
              Sint[e][(((size_t)(3 * r + c)) * N + kk) * n2 + q * n1 + p] = s;
            }
        }
      }
  }
  // Master-outward sub-face vectors of side s: the face's n s polynomial integrated over each sub-face.
  void ensure_fv_side(int s) {
    if (!Sbnd[s].empty()) return;
    ensure_side(s);
    Sbnd[s].assign(3 * (size_t)n2, 0.0);
    for (int c = 0; c < 3; ++c)
      for (int q = 0; q < n1; ++q)
        for (int p = 0; p < n1; ++p) {
          double v = 0.0;
          for (int b2 = 0; b2 < n1; ++b2)
            for (int a2 = 0; a2 < n1; ++a2) v += Bsub[p * n1 + a2] * Bsub[q * n1 + b2] * nvec[s][(size_t)c * n2 + b2 * n1 + a2];
          Sbnd[s][(size_t)c * n2 + q * n1 + p] = v;
        }
  }
  // Integral means (over the sub-cells) of the nodal state Ue [5][n3]: mean = B3 (J U) / V.
  template <class T> void dg_to_fv(int e, const T* Ue, T* out) {
    ensure_fv_geom(e);
    std::vector<T> ju(n3), m(n3);
    for (int v = 0; v < 5; ++v) {
      for (int t = 0; t < n3; ++t) ju[t] = Jdet[e][t] * Ue[(size_t)v * n3 + t];
      apply3(Bsub, ju.data(), m.data());
      for (int t = 0; t < n3; ++t) out[(size_t)v * n3 + t] = m[t] / Vsub[e][t];
    }
  }
  // Inverse: the nodal state whose sub-cell means are Ue: J U = B3^-1 (V mean).
  template <class T> void fv_to_dg(int e, const T* Ue, T* out) {
    ensure_fv_geom(e);
    std::vector<T> vm(n3), ju(n3);
    for (int v = 0; v < 5; ++v) {
      for (int t = 0; t < n3; ++t) vm[t] = Vsub[e][t] * Ue[(size_t)v * n3 + t];
      apply3(Bsubinv, vm.data(), ju.data());
      for (int t = 0; t < n3; ++t) out[(size_t)v * n3 + t] = ju[t] / Jdet[e][t];
    }
  }
  bool side_fv(int s) const { return C.fv && (fvmask[sideElem[2 * s]] || fvmask[sideElem[2 * s + 1]]); }
  template <class T> static T minmod(const T& a, const T& b) {
    if (val(a) * val(b) <= 0.0) return T(0.0);
    return std::fabs(val(a)) <= std::fabs(val(b)) ? a : b;
  }
  template <class T> void cons_to_w(const T* U, T* W) const {
    T rho, u[3], p; prim(U, rho, u, p);
    W[0] = rho; W[1] = u[0]; W[2] = u[1]; W[3] = u[2]; W[4] = p;
  }
  template <class T> void w_to_cons(const T* W, T* U) const {
    U[0] = W[0];
    for (int d = 0; d < 3; ++d) U[1 + d] = W[0] * W[1 + d];
    U[4] = W[4] / (C.gamma - 1.0) + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  }
  // Rusanov flux through the area vector S (not normalised) between primitive states.
  template <class T> void rusanov_w(const T* WL, const T* WR, const double* S, T* F) const {
    T UL[5], UR[5], FL[5], FR[5];
    w_to_cons(WL, UL); w_to_cons(WR, UR);
    flux_adv(UL, S, FL); flux_adv(UR, S, FR);
    const double sA = std::sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    const double nh[3] = {S[0] / sA, S[1] / sA, S[2] / sA};
    T cl = sqrt(C.gamma * WL[4] / WL[0]), cr = sqrt(C.gamma * WR[4] / WR[0]);
    T unl = WL[1] * nh[0] + WL[2] * nh[1] + WL[3] * nh[2];
    T unr = WR[1] * nh[0] + WR[2] * nh[1] + WR[3] * nh[2];
    T lmax = maxv(T(absv(unl) + cl), T(absv(unr) + cr));
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * (lmax * sA) * (UR[v] - UL[v]);
  }
  template <class T> void ensure_fv_caches(Work<T>& W) const {
    if (W.fvc.empty()) W.fvc.assign(nElems, {});
    if (C.physics == 1 && W.fvg.empty()) W.fvg.assign(nElems, {});
  }
  // Sub-cell means of element e ([5][n3]): its state if FV, else its DG state's means (cached).
  template <class T> const std::vector<T>& elem_means(const T* U, int e, Work<T>& W) {
    std::vector<T>& c = W.fvc[e];
    if (c.empty()) {
      c.assign(5 * (size_t)n3, T(0.0));
      std::vector<T> Ue(5 * (size_t)n3);
      for (int v = 0; v < 5; ++v)
        for (int t = 0; t < n3; ++t) Ue[(size_t)v * n3 + t] = U[uidx(v, e, t)];
      if (fvmask[e]) c = Ue;
      else dg_to_fv(e, Ue.data(), c.data());
    }
    return c;
  }
  // Primitive mean of the sub-cell in layer `layer` (0 = at the face) under face f, face-local (pp, qq).
  template <class T> void layer_w(const std::vector<T>& M, int f, int pp, int qq, int layer, T* W) const {
    const int l = (f % 2) ? C.N - layer : layer;
    int i, j, k; vol_ijk(f, pp, qq, l, i, j, k);
    T Uc[5];
    for (int v = 0; v < 5; ++v) Uc[v] = M[(size_t)v * n3 + node(i, j, k)];
    cons_to_w(Uc, W);
  }
  // Lifted variables q = (u, v, w, T) of a primitive state.
  template <class T> void w_to_q(const T* W, T* q) const {
    q[0] = W[1]; q[1] = W[2]; q[2] = W[3]; q[3] = W[4] / (W[0] * C.R);
  }

  // ---- Navier-Stokes on FV sub-cells (a reading; the paper names the FV
  // sub-cell scheme without its viscous terms).  BR1's ingredients carried to
  // the sub-cells: Green-Gauss gradients with central face values of
  // q = (u, v, w, T), and the central mean of both sides' viscous fluxes on
  // every sub-face.  Across an element face the other side is the neighbour's
  // layer-0 sub-cell: its state means, and its gradient (Green-Gauss if FV,
  // the sub-cell mean of its lifted gradient if DG).

  // Sub-cell gradients of element e ([12][n3], component 3a+d = dq_a/dx_d):
  //   FV element: g_s = (1/V_s) sum over its six sub-faces of 1/2 (q_s + q_s') S_out;
  //   DG element: the sub-cell means of its lifted gradient, B3(J g)/V.
  template <class T> const std::vector<T>& elem_grad(const T* U, int e, Work<T>& W) {
    std::vector<T>& g = W.fvg[e];
    if (!g.empty()) return g;
    ensure_fv_geom(e);
    g.assign(12 * (size_t)n3, T(0.0));
    if (!fvmask[e]) {
      lift_elem(U, e, W);
      std::vector<T> jg(n3), m(n3);
      for (int c = 0; c < 12; ++c) {
        for (int t = 0; t < n3; ++t) jg[t] = Jdet[e][t] * W.g[e][(size_t)c * n3 + t];
        apply3(Bsub, jg.data(), m.data());
        for (int t = 0; t < n3; ++t) g[(size_t)c * n3 + t] = m[t] / Vsub[e][t];
      }
      return g;
    }
    const int N = C.N;
    const std::vector<T>& M = elem_means(U, e, W);
    std::vector<T> q(4 * (size_t)n3);
    for (int t = 0; t < n3; ++t) {
      T Uc[5], Wc[5], qc[4];
      for (int v = 0; v < 5; ++v) Uc[v] = M[(size_t)v * n3 + t];
      cons_to_w(Uc, Wc); w_to_q(Wc, qc);
      for (int a = 0; a < 4; ++a) q[(size_t)a * n3 + t] = qc[a];
    }
    auto add = [&](int t, const T* qf, const double* S, double sg) {
      for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) g[(size_t)(3 * a + d) * n3 + t] += sg * (qf[a] * S[d]);
    };
    for (int r = 0; r < 3; ++r)
      for (int qq = 0; qq < n1; ++qq)
        for (int pp = 0; pp < n1; ++pp) {
          // interior sub-faces between layers kk and kk+1 along r
          for (int kk = 0; kk < N; ++kk) {
            int i, j, k; vol_ijk(2 * r, pp, qq, kk, i, j, k);
            int i2, j2, k2; vol_ijk(2 * r, pp, qq, kk + 1, i2, j2, k2);
            const int ta = node(i, j, k), tb = node(i2, j2, k2);
            double S[3];
            for (int c = 0; c < 3; ++c) S[c] = Sint[e][(((size_t)(3 * r + c)) * N + kk) * n2 + qq * n1 + pp];
            T qf[4];
            for (int a = 0; a < 4; ++a) qf[a] = 0.5 * (q[(size_t)a * n3 + ta] + q[(size_t)a * n3 + tb]);
            add(ta, qf, S, 1.0);
            add(tb, qf, S, -1.0);
          }
          // the two element faces normal to r
          for (int end = 0; end < 2; ++end) {
            const int f = 2 * r + end, s = elemSide[e * 6 + f], m = elemSlot[e * 6 + f];
            int p = pp, qm = qq;
            if (m == 1) orient_inv(sideOrient[s], C.N, pp, qq, p, qm);
            ensure_fv_side(s);
            double S[3];
            for (int c = 0; c < 3; ++c) S[c] = (m == 0 ? 1.0 : -1.0) * Sbnd[s][(size_t)c * n2 + qm * n1 + p];
            int i, j, k; vol_ijk(f, pp, qq, end ? N : 0, i, j, k);
            const int t = node(i, j, k);
            T Wg[5], qg[4], qf[4];
            ghost_w(U, e, f, pp, qq, W, Wg);
            w_to_q(Wg, qg);
            for (int a = 0; a < 4; ++a) qf[a] = 0.5 * (q[(size_t)a * n3 + t] + qg[a]);
            add(t, qf, S, 1.0);
          }
        }
    for (size_t c = 0; c < 12; ++c)
      for (int t = 0; t < n3; ++t) g[c * n3 + t] = g[c * n3 + t] / Vsub[e][t];
    return g;
  }
  // Gradient of the sub-cell in layer 0 under face f of element e, face-local (pp, qq).
  template <class T> void layer_g(const T* U, int e, int f, int pp, int qq, Work<T>& W, T* g) {
    const std::vector<T>& G = elem_grad(U, e, W);
    int i, j, k; vol_ijk(f, pp, qq, (f % 2) ? C.N : 0, i, j, k);
    for (int c = 0; c < 12; ++c) g[c] = G[(size_t)c * n3 + node(i, j, k)];
  }
  // Viscous flux G(W, g) . S of a primitive state and a gradient through the area vector S.
  template <class T> void visc_w(const T* Wp, const T* g, const double* S, T* F) const {
    T Uc[5];
    w_to_cons(Wp, Uc);
    for (int v = 0; v < 5; ++v) F[v] = T(0.0);
    for (int n = 0; n < 3; ++n) {
      T Gn[5]; flux_visc(Uc, g, n, Gn);
      for (int v = 0; v < 5; ++v) F[v] += Gn[v] * S[n];
    }
  }

  // Master-outward sub-face fluxes [5][n2] of an FV side (master sub-face
  // indexing): Rusanov between the MUSCL-reconstructed states, minus (Navier-
  // Stokes) the central mean of both layer-0 sub-cells' viscous fluxes.
  // Both sides' layer-0 means W0 and reconstructed face states Wf at master
  // sub-face (p, q) of an FV side: Wf = W0 + 1/2 minmod(W0 - W1, W0' - W0),
  // W1 the layer-1 mean, W0' the other side's layer-0 mean.
  template <class T> void side_face_states(const T* U, int s, int p, int q, Work<T>& W, T W0[2][5], T Wf[2][5]) {
    T W1[2][5];
    for (int m = 0; m < 2; ++m) {
      const int e = sideElem[2 * s + m], f = sideLoc[2 * s + m];
      int pp = p, qq = q;
      if (m == 1) orient_fwd(sideOrient[s], C.N, p, q, pp, qq);
      const std::vector<T>& M = elem_means(U, e, W);
      layer_w(M, f, pp, qq, 0, W0[m]); layer_w(M, f, pp, qq, 1, W1[m]);
    }
    for (int m = 0; m < 2; ++m)
      for (int v = 0; v < 5; ++v) {
        const T sg = minmod(T(W0[m][v] - W1[m][v]), T(W0[1 - m][v] - W0[m][v]));
        Wf[m][v] = W0[m][v] + 0.5 * sg;
      }
  }
  template <class T> void side_flux_fv(const T* U, int s, Work<T>& W, std::vector<T>& F) {
    ensure_fv_side(s);
    F.assign(5 * (size_t)n2, T(0.0));
    for (int q = 0; q < n1; ++q)
      for (int p = 0; p < n1; ++p) {
        T W0[2][5], Wf[2][5], G0[2][12];
        side_face_states(U, s, p, q, W, W0, Wf);
        if (C.physics == 1)
          for (int m = 0; m < 2; ++m) {
            int pp = p, qq = q;
            if (m == 1) orient_fwd(sideOrient[s], C.N, p, q, pp, qq);
            layer_g(U, sideElem[2 * s + m], sideLoc[2 * s + m], pp, qq, W, G0[m]);
          }
        const double S[3] = {Sbnd[s][q * n1 + p], Sbnd[s][(size_t)n2 + q * n1 + p], Sbnd[s][2 * (size_t)n2 + q * n1 + p]};
        T Fs[5]; rusanov_w(Wf[0], Wf[1], S, Fs);
        if (C.physics == 1) {
          T GL[5], GR[5];
          visc_w(W0[0], G0[0], S, GL); visc_w(W0[1], G0[1], S, GR);
          for (int v = 0; v < 5; ++v) Fs[v] -= 0.5 * (GL[v] + GR[v]);
        }
        for (int v = 0; v < 5; ++v) F[(size_t)v * n2 + q * n1 + p] = Fs[v];
      }
  }
  // DG side of an FV face: the nodal flux polynomial whose sub-face integrals are F (master indexing).
  template <class T> void fv_face_to_nodal(const std::vector<T>& F, std::vector<T>& Phi) const {
    Phi.assign(5 * (size_t)n2, T(0.0));
    for (int v = 0; v < 5; ++v)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          T s(0.0);
          for (int q = 0; q < n1; ++q)
            for (int p = 0; p < n1; ++p) s += Bsubinv[i * n1 + p] * Bsubinv[j * n1 + q] * F[(size_t)v * n2 + q * n1 + p];
          Phi[(size_t)v * n2 + j * n1 + i] = s;
        }
  }
  // Primitive layer-0 mean of the neighbour across face f of element e, at own face-local (pp, qq).
  template <class T> void ghost_w(const T* U, int e, int f, int pp, int qq, Work<T>& W, T* Wout) {
    const int s = elemSide[e * 6 + f], m = elemSlot[e * 6 + f];
    int p = pp, q = qq;
    if (m == 1) orient_inv(sideOrient[s], C.N, pp, qq, p, q);
    const int o = 1 - m;
    const int eo = sideElem[2 * s + o], fo = sideLoc[2 * s + o];
    int po = p, qo = q;
    if (o == 1) orient_fwd(sideOrient[s], C.N, p, q, po, qo);
    layer_w(elem_means(U, eo, W), fo, po, qo, 0, Wout);
  }
  // Lifting of a DG element on an FV face: the FV neighbour's q at the own
  // face node (pp, qq) is the face polynomial whose reference sub-face means
  // are the q of the FV side's reconstructed face states (those the face
  // flux uses): q = h^2 (B^-1 x B^-1) q_f, h = 2/(N+1).  B integrates over the
  // sub-intervals, so this is the degree-N polynomial with those means; for
  // a linear field it is the field itself.
  template <class T> void fv_face_q(const T* U, int e, int f, int pp, int qq, Work<T>& W, T* qf) {
    const double h = 2.0 / n1;
    const int s = elemSide[e * 6 + f], m = elemSlot[e * 6 + f];
    for (int a = 0; a < 4; ++a) qf[a] = T(0.0);
    for (int q2 = 0; q2 < n1; ++q2)
      for (int p2 = 0; p2 < n1; ++p2) {
        int p = p2, q = q2;
        if (m == 1) orient_inv(sideOrient[s], C.N, p2, q2, p, q);
        T W0[2][5], Wf[2][5], qg[4];
        side_face_states(U, s, p, q, W, W0, Wf);
        w_to_q(Wf[1 - m], qg);
        const double c = h * h * Bsubinv[pp * n1 + p2] * Bsubinv[qq * n1 + q2];
        for (int a = 0; a < 4; ++a) qf[a] += c * qg[a];
      }
  }
  // FV residual of element e: dmean/dt = -(1/V) sum of outward sub-face fluxes
  // (advective minus viscous).
  template <class T> void residual_fv(const T* U, int e, Work<T>& Wk, std::vector<std::vector<T>>& sfv, T* Ut) {
    ensure_fv_geom(e);
    const int N = C.N;
    const std::vector<T>& M = elem_means(U, e, Wk);
    const std::vector<T>* Gp = C.physics == 1 ? &elem_grad(U, e, Wk) : nullptr;
    std::vector<T> R(5 * (size_t)n3, T(0.0));
    for (int r = 0; r < 3; ++r)
      for (int qq = 0; qq < n1; ++qq)
        for (int pp = 0; pp < n1; ++pp) {
          // cells -1..N+1 along the line (ghosts from the neighbours)
          std::vector<std::array<T, 5>> W(n1 + 2);
          for (int l = 0; l < n1; ++l) {
            int i, j, k; vol_ijk(2 * r, pp, qq, l, i, j, k);
            T Uc[5];
            for (int v = 0; v < 5; ++v) Uc[v] = M[(size_t)v * n3 + node(i, j, k)];
            cons_to_w(Uc, W[l + 1].data());
          }
          ghost_w(U, e, 2 * r, pp, qq, Wk, W[0].data());
          ghost_w(U, e, 2 * r + 1, pp, qq, Wk, W[n1 + 1].data());
          std::vector<std::array<T, 5>> sg(n1);
          for (int l = 0; l < n1; ++l)
            for (int v = 0; v < 5; ++v) sg[l][v] = minmod(T(W[l + 2][v] - W[l + 1][v]), T(W[l + 1][v] - W[l][v]));
          for (int kk = 0; kk < N; ++kk) {
            T WL[5], WR[5];
            for (int v = 0; v < 5; ++v) { WL[v] = W[kk + 1][v] + 0.5 * sg[kk][v]; WR[v] = W[kk + 2][v] - 0.5 * sg[kk + 1][v]; }
            double S[3];
            for (int c = 0; c < 3; ++c) S[c] = Sint[e][(((size_t)(3 * r + c)) * N + kk) * n2 + qq * n1 + pp];
            T F[5]; rusanov_w(WL, WR, S, F);
            int i, j, k; vol_ijk(2 * r, pp, qq, kk, i, j, k);
            int i2, j2, k2; vol_ijk(2 * r, pp, qq, kk + 1, i2, j2, k2);
            if (Gp) {
              // central viscous flux between the two sub-cells (means and their gradients)
              T ga[12], gb[12], GL[5], GR[5];
              for (int c = 0; c < 12; ++c) {
                ga[c] = (*Gp)[(size_t)c * n3 + node(i, j, k)];
                gb[c] = (*Gp)[(size_t)c * n3 + node(i2, j2, k2)];
              }
              visc_w(W[kk + 1].data(), ga, S, GL); visc_w(W[kk + 2].data(), gb, S, GR);
              for (int v = 0; v < 5; ++v) F[v] -= 0.5 * (GL[v] + GR[v]);
            }
            for (int v = 0; v < 5; ++v) {
              R[(size_t)v * n3 + node(i, j, k)] -= F[v];
              R[(size_t)v * n3 + node(i2, j2, k2)] += F[v];
            }
          }
          // the element's two faces normal to r: outward sub-face fluxes
          for (int end = 0; end < 2; ++end) {
            const int f = 2 * r + end, s = elemSide[e * 6 + f], m = elemSlot[e * 6 + f];
            int p = pp, q = qq;
            if (m == 1) orient_inv(sideOrient[s], C.N, pp, qq, p, q);
            int i, j, k; vol_ijk(f, pp, qq, end ? N : 0, i, j, k);
            for (int v = 0; v < 5; ++v) {
              const T Fo = (m == 0) ? sfv[s][(size_t)v * n2 + q * n1 + p] : T(-sfv[s][(size_t)v * n2 + q * n1 + p]);
              R[(size_t)v * n3 + node(i, j, k)] -= Fo;
            }
          }
        }
    for (int v = 0; v < 5; ++v)
      for (int t = 0; t < n3; ++t) Ut[oidx(v, e, t)] = R[(size_t)v * n3 + t] / Vsub[e][t];
  }

  // Persson-Peraire indicator: log10 of the share of the highest modes
  // (max(i,j,k) = N in the orthonormal Legendre basis) in the energy of rho.
  double indicator(const double* U, int e) {
    std::vector<double> Ue(5 * (size_t)n3), Ud(5 * (size_t)n3);
    for (int v = 0; v < 5; ++v)
      for (int t = 0; t < n3; ++t) Ue[(size_t)v * n3 + t] = U[uidx(v, e, t)];
    if (C.fv && fvmask[e]) fv_to_dg(e, Ue.data(), Ud.data());
    else Ud = Ue;
    std::vector<double> mod(n3);
    apply3(Vleginv, Ud.data(), mod.data());
    double Eall = 0.0, Etop = 0.0;
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          const double c2 = mod[node(i, j, k)] * mod[node(i, j, k)];
          Eall += c2;
          if (i == C.N || j == C.N || k == C.N) Etop += c2;
        }
    return std::log10(std::max(Etop / Eall, 1e-30));
  }
  // Element types to `newmask`, converting U (and dU) of the elements that change.
  void fv_switch(double* U, double* dU, const int* newmask) {
    std::vector<double> a(5 * (size_t)n3), b(5 * (size_t)n3);
    for (int e = 0; e < nElems; ++e) {
      if ((newmask[e] != 0) == (fvmask[e] != 0)) continue;
      for (double* X : {U, dU}) {
        if (!X) continue;
        for (int v = 0; v < 5; ++v)
          for (int t = 0; t < n3; ++t) a[(size_t)v * n3 + t] = X[uidx(v, e, t)];
        if (newmask[e]) dg_to_fv(e, a.data(), b.data());
        else fv_to_dg(e, a.data(), b.data());
        for (int v = 0; v < 5; ++v)
          for (int t = 0; t < n3; ++t) X[uidx(v, e, t)] = b[(size_t)v * n3 + t];
      }
      fvmask[e] = newmask[e] ? 1 : 0;
    }
  }

  // Hybridised SBP operator of one line with nodes 0..N and the two faces
  // (N+1: xi = -1, N+2: xi = +1), E = [Lm; Lp] the interpolation to the
  // faces, Bf = diag(-1, +1):
  //   Q_h = 1/2 [[Q - Q^T, E^T Bf], [-Bf E, Bf]],   Q = M D.
  std::vector<double> hybrid_operator() const {
    const int nh = n1 + 2;
    std::vector<double> Qh((size_t)nh * nh, 0.0);
    const double Bf[2] = {-1.0, 1.0};
    const std::vector<double>* E[2] = {&B.Lm, &B.Lp};
    for (int i = 0; i < n1; ++i)
      for (int j = 0; j < n1; ++j) Qh[i * nh + j] = 0.5 * (B.w[i] * B.D[i * n1 + j] - B.w[j] * B.D[j * n1 + i]);
    for (int f = 0; f < 2; ++f) {
      for (int i = 0; i < n1; ++i) {
        Qh[i * nh + n1 + f] = 0.5 * (*E[f])[i] * Bf[f];
        Qh[(n1 + f) * nh + i] = -0.5 * Bf[f] * (*E[f])[i];
      }
      Qh[(n1 + f) * nh + n1 + f] = 0.5 * Bf[f];
    }
    return Qh;
  }

  // Volume contribution of one line of element e along direction r through
  // the hybridised operator (Chan, Del Rey Fernandez & Carpenter 2019):
  //   M dU/dt += -[I, E^T] 2 (Q_h o F) 1 - E^T Bf (f* - f(u~_f)),
  // F_mn = F#(u~_m, u~_n) . (Ja_m + Ja_n)/2 over the hybrid node set, with
  // u~ = U at the volume nodes, u~_f = u(E v(U)) at the faces, and the face
  // metric Ja_f = E Ja^r.  This adds everything but the f* part, which the
  // surface term supplies.
  template <class T> void hybrid_line(const T* U, int e, int r, int pp, int qq, std::vector<T>& V) {
    const int nh = n1 + 2;
    const std::vector<double> Qh = hybrid_operator();
    const std::vector<double>& M = Ja[e];
    const std::vector<double>* E[2] = {&B.Lm, &B.Lp};
    std::vector<int> tl(n1);
    for (int l = 0; l < n1; ++l) {
      int i, j, k; vol_ijk(2 * r, pp, qq, l, i, j, k);
      tl[l] = node(i, j, k);
    }
    std::vector<T> Uh((size_t)5 * nh);
    std::vector<double> Jh((size_t)3 * nh, 0.0);
    for (int l = 0; l < n1; ++l) {
      for (int v = 0; v < 5; ++v) Uh[(size_t)v * nh + l] = U[uidx(v, e, tl[l])];
      for (int c = 0; c < 3; ++c) Jh[(size_t)c * nh + l] = M[(size_t)(3 * r + c) * n3 + tl[l]];
    }
    for (int f = 0; f < 2; ++f) {
      T vf[5];
      for (int v = 0; v < 5; ++v) vf[v] = T(0.0);
      for (int l = 0; l < n1; ++l) {
        T Ul[5], x[5];
        for (int v = 0; v < 5; ++v) Ul[v] = Uh[(size_t)v * nh + l];
        entropy_vars(Ul, x);
        for (int v = 0; v < 5; ++v) vf[v] += (*E[f])[l] * x[v];
        for (int c = 0; c < 3; ++c) Jh[(size_t)c * nh + n1 + f] += (*E[f])[l] * Jh[(size_t)c * nh + l];
      }
      T uf[5];
      cons_from_entropy(vf, uf);
      for (int v = 0; v < 5; ++v) Uh[(size_t)v * nh + n1 + f] = uf[v];
    }
    // r_h = 2 (Q_h o F) 1
    std::vector<T> rh((size_t)5 * nh, T(0.0));
    for (int m = 0; m < nh; ++m)
      for (int n = 0; n < nh; ++n) {
        const double q = Qh[m * nh + n];
        if (q == 0.0) continue;
        T Ua[5], Ub[5];
        for (int v = 0; v < 5; ++v) { Ua[v] = Uh[(size_t)v * nh + m]; Ub[v] = Uh[(size_t)v * nh + n]; }
        double nv[3];
        for (int c = 0; c < 3; ++c) nv[c] = 0.5 * (Jh[(size_t)c * nh + m] + Jh[(size_t)c * nh + n]);
        T F[5]; flux_twopoint(Ua, Ub, nv, F);
        for (int v = 0; v < 5; ++v) rh[(size_t)v * nh + m] += 2.0 * q * F[v];
      }
    const double Bf[2] = {-1.0, 1.0};
    for (int a = 0; a < n1; ++a)
      for (int v = 0; v < 5; ++v) {
        T acc = rh[(size_t)v * nh + a];
        for (int f = 0; f < 2; ++f) acc += (*E[f])[a] * rh[(size_t)v * nh + n1 + f];
        V[(size_t)v * n3 + tl[a]] -= acc / B.w[a];
      }
    // the f(u~_f) part of the surface correction
    for (int f = 0; f < 2; ++f) {
      T uf[5];
      for (int v = 0; v < 5; ++v) uf[v] = Uh[(size_t)v * nh + n1 + f];
      const double nv[3] = {Jh[n1 + f], Jh[(size_t)nh + n1 + f], Jh[2 * (size_t)nh + n1 + f]};
      T Ff[5]; flux_adv(uf, nv, Ff);
      for (int a = 0; a < n1; ++a)
        for (int v = 0; v < 5; ++v) V[(size_t)v * n3 + tl[a]] += (*E[f])[a] * Bf[f] * Ff[v] / B.w[a];
    }
  }

  template <class T> void rhs(const T* U, T* Ut, double t, const std::vector<int>& elist) {
    Work<T> W;
    W.tr.assign(nSides, {}); W.gtr.assign(nSides, {}); W.g.assign(nElems, {});
    std::vector<int> el = elist;
    if (el.empty()) { el.resize(nElems); for (int e = 0; e < nElems; ++e) el[e] = e; }
    std::vector<std::vector<T>> sflux(nSides);
    std::vector<std::vector<T>> sfv(C.fv ? nSides : 0);
    if (C.fv) ensure_fv_caches(W);
    for (int e : el) {
      if (C.physics == 1 && !(C.fv && fvmask[e])) lift_elem(U, e, W);
      for (int f = 0; f < 6; ++f) {
        int s = elemSide[e * 6 + f];
        if (C.fv && side_fv(s)) {
          // FV face: sub-face fluxes; the DG side takes their face polynomial
          if (sfv[s].empty()) { side_flux_fv(U, s, W, sfv[s]); fv_face_to_nodal(sfv[s], sflux[s]); }
        } else if (sflux[s].empty()) {
          side_flux(U, s, W, sflux[s]);
        }
      }
    }
    for (int e : el) {
      if (C.fv && fvmask[e]) residual_fv(U, e, W, sfv, Ut);
      else residual_elem(U, e, W, sflux, Ut, t);
    }
  }

  template <class T> void lift_all(const T* U, T* gout) {
    Work<T> W;
    W.tr.assign(nSides, {}); W.gtr.assign(nSides, {}); W.g.assign(nElems, {});
    for (int e = 0; e < nElems; ++e) {
      lift_elem(U, e, W);
      for (size_t c = 0; c < 12; ++c)
        for (int t = 0; t < n3; ++t) gout[(c * nElems + e) * n3 + t] = W.g[e][c * n3 + t];
    }
  }

  // Low-storage RK (LSERK4(5) or LSERK4-14), 2N-storage, per stage s:
  // dU <- A_s dU + dt R(U, t + c_s dt); U <- U + B_s dU.
  template <class T> void lserk(T* U, int nsteps, double dt, double t0) {
    const size_t n = (size_t)5 * nElems * n3;
    std::vector<T> dU(n, T(0.0)), R(n);
    std::vector<int> all;
    double t = t0;
    for (int step = 0; step < nsteps; ++step) {
      for (int s = 0; s < nstages; ++s) {
        rhs(U, R.data(), t + lsC[s] * dt, all);
        for (size_t i = 0; i < n; ++i) {
          dU[i] = lsA[s] * dU[i] + dt * R[i];
          U[i] = U[i] + lsB[s] * dU[i];
        }
      }
      t += dt;
    }
  }

  // Transposed residual Jacobian applied to lam: out = (dR/dU)^T lam at U.
  // R(U) is recorded on the tape (one node per input, then one per
  // operation) and the tape is swept back from the outputs' seeds lam.
  void rhs_vjp(const double* U, const double* lam, double* out, double t) {
    const size_t n = (size_t)5 * nElems * n3;
    for (int e = 0; e < nElems; ++e) ensure_geom(e);
    for (int s = 0; s < nSides; ++s) ensure_side(s);
    g_tape.clear();
    std::vector<Rev> X(n), Y(n);
    for (size_t i = 0; i < n; ++i) X[i] = Rev::input(U[i]);   // tape nodes 0..n-1
    std::vector<int> all;
    rhs<Rev>(X.data(), Y.data(), t, all);
    std::vector<double> adj(g_tape.size(), 0.0);
    for (size_t i = 0; i < n; ++i)
      if (Y[i].i >= 0) adj[Y[i].i] += lam[i];
    g_tape.sweep(adj);
    for (size_t i = 0; i < n; ++i) out[i] = adj[i];
    g_tape.clear();
  }

  // Gradient of E_k at U (scaled by `scale`), from the tape of kinetic_energy.
  void kinetic_energy_grad(const double* U, double rho0U0sq, double* grad) {
    const size_t n = (size_t)5 * nElems * n3;
    for (int e = 0; e < nElems; ++e) ensure_geom(e);
    g_tape.clear();
    std::vector<Rev> X(n);
    for (size_t i = 0; i < n; ++i) X[i] = Rev::input(U[i]);
    Rev Ek = kinetic_energy<Rev>(X.data(), rho0U0sq);
    std::vector<double> adj(g_tape.size(), 0.0);
    if (Ek.i >= 0) adj[Ek.i] = 1.0;
    g_tape.sweep(adj);
    for (size_t i = 0; i < n; ++i) grad[i] = adj[i];
    g_tape.clear();
  }

  // Reverse sweep of nsteps steps of the low-storage scheme started from U0.
  // On entry lamU = dJ/dU at the final state, on exit dJ/dU0.  A stage reads
  // Y_s (the stage input), dU <- A_s dU + dt R(Y_s, t + c_s dt) and
  // Y_{s+1} = Y_s + B_s dU; its adjoint, taken for s = S-1 down to 0 with
  // lamdU = 0 at the end of each step (dU enters a step multiplied by
  // A_0 = 0), is
  //   lamdU += B_s lamU;   lamU += dt (dR/dU(Y_s))^T lamdU;   lamdU <- A_s lamdU.
  // The step states are recomputed forward and kept; each step's stage
  // inputs are recomputed from its step state.
  void lserk_adjoint(const double* U0, double* lamU, int nsteps, double dt, double t0) {
    const size_t n = (size_t)5 * nElems * n3;
    std::vector<std::vector<double>> Ustep(nsteps);
    std::vector<double> U(U0, U0 + n);
    for (int step = 0; step < nsteps; ++step) {
      Ustep[step] = U;
      lserk<double>(U.data(), 1, dt, t0 + step * dt);
    }
    std::vector<std::vector<double>> Y(nstages, std::vector<double>(n));
    std::vector<double> dU(n), R(n), lamdU(n), vj(n);
    std::vector<int> all;
    for (int step = nsteps - 1; step >= 0; --step) {
      const double ts = t0 + step * dt;
      // stage inputs of this step
      Y[0] = Ustep[step];
      std::fill(dU.begin(), dU.end(), 0.0);
      for (int s = 0; s + 1 < nstages; ++s) {
        rhs<double>(Y[s].data(), R.data(), ts + lsC[s] * dt, all);
        for (size_t i = 0; i < n; ++i) {
          dU[i] = lsA[s] * dU[i] + dt * R[i];
          Y[s + 1][i] = Y[s][i] + lsB[s] * dU[i];
        }
      }
      std::fill(lamdU.begin(), lamdU.end(), 0.0);
      for (int s = nstages - 1; s >= 0; --s) {
        for (size_t i = 0; i < n; ++i) lamdU[i] += lsB[s] * lamU[i];
        rhs_vjp(Y[s].data(), lamdU.data(), vj.data(), ts + lsC[s] * dt);
        for (size_t i = 0; i < n; ++i) {
          lamU[i] += dt * vj[i];
          lamdU[i] = lsA[s] * lamdU[i];
        }
      }
    }
  }

  // Integral kinetic energy (TGV section) with collocated quadrature:
  // E_k = sum w_i w_j w_k J |m|^2/rho / (2 rho0 U0^2 |Omega|),  |Omega| = sum w J.
  template <class T> T kinetic_energy(const T* U, double rho0U0sq) {
    T acc(0.0);
    double vol = 0.0;
    for (int e = 0; e < nElems; ++e) {
      ensure_geom(e);
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            int tt = node(i, j, k);
            double wJ = B.w[i] * B.w[j] * B.w[k] * Jdet[e][tt];
            T rho = U[uidx(0, e, tt)];
            T m2 = U[uidx(1, e, tt)] * U[uidx(1, e, tt)] + U[uidx(2, e, tt)] * U[uidx(2, e, tt)] +
                   U[uidx(3, e, tt)] * U[uidx(3, e, tt)];
            acc += wJ * (m2 / rho);
            vol += wJ;
          }
    }
    return acc / (2.0 * rho0U0sq * vol);
  }

  // Fixed time step.  The paper fixes CFL = 0.9 for the advective and the
  // viscous restriction but prints no formula.  Reading used here:
  //   dt_a = cfl * min(2/(N+1), 8/(N+1)^2) / max_node sum_r (|Ja^r.u| + c |Ja^r|)/J
  //   dt_v = cfl * 32/(N+1)^4 / max_node (mu/rho) max(4/3, gamma/Pr) sum_r |Ja^r|^2/J^2
  // the N-scalings follow the growth of the DG spectral radius (N^2 for the
  // advective, N^4 for the viscous operator); the constants keep LSERK4(5)
  // linearly stable for N = 1..7 at cfl = 0.9 (checked in the test suite).
  double timestep(const double* U, double cfl) {
    double amax = 0.0, vmax = 0.0;
    for (int e = 0; e < nElems; ++e) {
      ensure_geom(e);
      for (int tt = 0; tt < n3; ++tt) {
        double Ul[5];
        for (int v = 0; v < 5; ++v) Ul[v] = U[uidx(v, e, tt)];
        double rho, u[3], p; prim(Ul, rho, u, p);
        double c = std::sqrt(C.gamma * p / rho);
        double J = Jdet[e][tt];
        double sa = 0.0, sv = 0.0;
        for (int r = 0; r < 3; ++r) {
          const double* M = &Ja[e][(size_t)(3 * r) * n3 + tt];
          double a0 = M[0], a1 = M[(size_t)n3], a2 = M[2 * (size_t)n3];
          double nrm2 = a0 * a0 + a1 * a1 + a2 * a2;
          sa += std::fabs(a0 * u[0] + a1 * u[1] + a2 * u[2]) + c * std::sqrt(nrm2);
          sv += nrm2;
        }
        amax = std::max(amax, sa / J);
        vmax = std::max(vmax, viscosity(p / (rho * C.R)) / rho * std::max(4.0 / 3.0, C.gamma / C.Pr) * sv / (J * J));
      }
    }
    // LSERK4-14: its stability region reaches 3.98 times further along the
    // DG spectrum (eigenvalues of the linearised operator), step scaled by 3.75
    const double n1 = C.N + 1.0;
    const double sc = cfl * (C.integrator == 1 ? 3.75 : 1.0);
    double dt = sc * std::min(2.0 / n1, 8.0 / (n1 * n1)) / amax;
    if (C.physics == 1 && vmax > 0.0) dt = std::min(dt, sc * 32.0 / (n1 * n1 * n1 * n1 * vmax));
    return dt;
  }
};

}  // namespace orc

using orc::Solver;

// ---------------------------------------------------------------------------
// C interface used by the test suite (through ctypes).
// icfg = {N, nodes, form, physics, twopoint, dissipation, mms, integrator, viscosity, hybrid, fv}
// dcfg = {gamma, mu, Pr, R, mms_A, mms_a, Tref, Ts}
// ---------------------------------------------------------------------------
extern "C" {

static thread_local std::string g_err;

const char* orc_last_error() { return g_err.c_str(); }

int orc_basis(int N, int type, double* x, double* w, double* D, double* Lm, double* Lp, double* DS) {
  orc::Basis B;
  if (!orc::make_basis(N, type, B)) return 1;
  int n = N + 1;
  for (int i = 0; i < n; ++i) { x[i] = B.x[i]; w[i] = B.w[i]; Lm[i] = B.Lm[i]; Lp[i] = B.Lp[i]; }
  for (int i = 0; i < n * n; ++i) { D[i] = B.D[i]; DS[i] = B.DS[i]; }
  return 0;
}

void* orc_create(const int* icfg, const double* dcfg, int nElems, int Ngeo, const double* Xgeo, int nSides,
                 const int* sideElem, const int* sideLoc, const int* sideOrient) {
  Solver* S = new Solver();
  S->C.N = icfg[0]; S->C.nodes = icfg[1]; S->C.form = icfg[2]; S->C.physics = icfg[3];
  S->C.twopoint = icfg[4]; S->C.dissipation = icfg[5]; S->C.mms = icfg[6]; S->C.integrator = icfg[7];
  S->C.viscosity = icfg[8]; S->C.hybrid = icfg[9]; S->C.fv = icfg[10];
  S->C.gamma = dcfg[0]; S->C.mu = dcfg[1]; S->C.Pr = dcfg[2]; S->C.R = dcfg[3];
  S->C.Tref = dcfg[6]; S->C.Ts = dcfg[7];
  S->C.mms_A = dcfg[4]; S->C.mms_a = dcfg[5];
  S->nElems = nElems; S->Ngeo = Ngeo; S->nSides = nSides;
  if (nElems <= 0 || Ngeo < 1 || nSides * 2 != nElems * 6) { g_err = "bad sizes"; delete S; return nullptr; }
  S->Xgeo.assign(Xgeo, Xgeo + (size_t)3 * nElems * (Ngeo + 1) * (Ngeo + 1) * (Ngeo + 1));
  S->sideElem.assign(sideElem, sideElem + 2 * (size_t)nSides);
  S->sideLoc.assign(sideLoc, sideLoc + 2 * (size_t)nSides);
  S->sideOrient.assign(sideOrient, sideOrient + nSides);
  if (!S->setup()) { g_err = S->err; delete S; return nullptr; }
  return S;
}

int orc_check_jacobians(void* h) {
  Solver* S = (Solver*)h;
  if (!S->check_jacobians()) { g_err = S->err; return 1; }
  return 0;
}

void orc_destroy(void* h) { delete (Solver*)h; }

void orc_lserk_coeffs(double* A, double* B, double* C) { orc::lserk_coeffs(A, B, C); }
int orc_rk_coeffs(int integrator, double* A, double* B, double* C) { return orc::rk_coeffs(integrator, A, B, C); }

// Node coordinates [3][nElems][n3], Jacobian [nElems][n3], metrics [9][nElems][n3].
void orc_geometry(void* h, double* xyz, double* J, double* Ja) {
  Solver* S = (Solver*)h;
  for (int e = 0; e < S->nElems; ++e) {
    S->ensure_geom(e);
    for (int t = 0; t < S->n3; ++t) {
      if (xyz) for (int d = 0; d < 3; ++d) xyz[((size_t)d * S->nElems + e) * S->n3 + t] = S->Xnode[e][(size_t)d * S->n3 + t];
      if (J) J[(size_t)e * S->n3 + t] = S->Jdet[e][t];
      if (Ja) for (int c = 0; c < 9; ++c) Ja[((size_t)c * S->nElems + e) * S->n3 + t] = S->Ja[e][(size_t)c * S->n3 + t];
    }
  }
}

// Geometry of a list of elements only, compact: xyz[3][nlist][n3], J[nlist][n3], Ja[9][nlist][n3].
int orc_geometry_sample(void* h, int nlist, const int* list, double* xyz, double* J, double* Ja) {
  Solver* S = (Solver*)h;
  for (int i = 0; i < nlist; ++i)
    if (list[i] < 0 || list[i] >= S->nElems) { g_err = "element out of range"; return 1; }
  for (int i = 0; i < nlist; ++i) {
    const int e = list[i];
    S->ensure_geom(e);
    for (int t = 0; t < S->n3; ++t) {
      if (xyz) for (int d = 0; d < 3; ++d) xyz[((size_t)d * nlist + i) * S->n3 + t] = S->Xnode[e][(size_t)d * S->n3 + t];
      if (J) J[(size_t)i * S->n3 + t] = S->Jdet[e][t];
      if (Ja) for (int c = 0; c < 9; ++c) Ja[((size_t)c * nlist + i) * S->n3 + t] = S->Ja[e][(size_t)c * S->n3 + t];
    }
  }
  return 0;
}

// Master-outward scaled normals n*s at face nodes: [3][nSides][n2].
void orc_face_normals(void* h, double* nv) {
  Solver* S = (Solver*)h;
  for (int s = 0; s < S->nSides; ++s) {
    S->ensure_side(s);
    for (int c = 0; c < 3; ++c)
      for (int t = 0; t < S->n2; ++t) nv[((size_t)c * S->nSides + s) * S->n2 + t] = S->nvec[s][(size_t)c * S->n2 + t];
  }
}

int orc_rhs(void* h, const double* U, double* Ut, double t) {
  Solver* S = (Solver*)h;
  std::vector<int> all;
  S->rhs<double>(U, Ut, t, all);
  return 0;
}

// Residual of a list of elements only; Ut is the full-size array, only the
// listed elements are written.
int orc_rhs_elems(void* h, const double* U, double* Ut, double t, int nlist, const int* list) {
  Solver* S = (Solver*)h;
  std::vector<int> el(list, list + nlist);
  for (int e : el)
    if (e < 0 || e >= S->nElems) { g_err = "element out of range"; return 1; }
  if (el.empty()) return 0;
  S->rhs<double>(U, Ut, t, el);
  return 0;
}

// Residual of a list of distinct elements into a compact array out[5][nlist][n3]
// (element list[i] at position i): the same arithmetic as orc_rhs_elems, with
// no full-size output.
int orc_rhs_sample(void* h, const double* U, double* out, double t, int nlist, const int* list) {
  Solver* S = (Solver*)h;
  std::vector<int> el(list, list + nlist);
  std::vector<int> pos(S->nElems, -1);
  for (int i = 0; i < nlist; ++i) {
    const int e = el[i];
    if (e < 0 || e >= S->nElems) { g_err = "element out of range"; return 1; }
    if (pos[e] >= 0) { g_err = "element listed twice"; return 1; }
    pos[e] = i;
  }
  if (el.empty()) return 0;
  S->outpos.swap(pos);
  S->outn = nlist;
  S->rhs<double>(U, out, t, el);
  S->outpos.clear();
  S->outn = 0;
  return 0;
}

// Lifted gradients [12][nElems][n3], component 3*a+d = d q_a / d x_d, q=(u,v,w,T).
int orc_lift(void* h, const double* U, double* g) {
  Solver* S = (Solver*)h;
  S->lift_all<double>(U, g);
  return 0;
}

// Tangent of the residual: dUt = (dR/dU) dU.
int orc_rhs_jvp(void* h, const double* U, const double* dU, double* Ut, double* dUt, double t) {
  Solver* S = (Solver*)h;
  size_t n = (size_t)5 * S->nElems * S->n3;
  std::vector<orc::Dual> X(n), Y(n);
  for (size_t i = 0; i < n; ++i) X[i] = orc::Dual(U[i], dU[i]);
  std::vector<int> all;
  S->rhs<orc::Dual>(X.data(), Y.data(), t, all);
  for (size_t i = 0; i < n; ++i) { if (Ut) Ut[i] = Y[i].v; dUt[i] = Y[i].d; }
  return 0;
}

int orc_lserk(void* h, double* U, int nsteps, double dt, double t0) {
  Solver* S = (Solver*)h;
  S->lserk<double>(U, nsteps, dt, t0);
  return 0;
}

// Tangent of a whole trajectory: U <- U(T), dU <- (dU(T)/dU(0)) dU.
int orc_lserk_jvp(void* h, double* U, double* dU, int nsteps, double dt, double t0) {
  Solver* S = (Solver*)h;
  size_t n = (size_t)5 * S->nElems * S->n3;
  std::vector<orc::Dual> X(n);
  for (size_t i = 0; i < n; ++i) X[i] = orc::Dual(U[i], dU[i]);
  S->lserk<orc::Dual>(X.data(), nsteps, dt, t0);
  for (size_t i = 0; i < n; ++i) { U[i] = X[i].v; dU[i] = X[i].d; }
  return 0;
}

double orc_kinetic_energy(void* h, const double* U, double rho0U0sq) {
  Solver* S = (Solver*)h;
  return S->kinetic_energy<double>(U, rho0U0sq);
}

// Directional derivative of E_k: returns dE_k/dU . dU.
double orc_kinetic_energy_jvp(void* h, const double* U, const double* dU, double rho0U0sq) {
  Solver* S = (Solver*)h;
  size_t n = (size_t)5 * S->nElems * S->n3;
  std::vector<orc::Dual> X(n);
  for (size_t i = 0; i < n; ++i) X[i] = orc::Dual(U[i], dU[i]);
  return S->kinetic_energy<orc::Dual>(X.data(), rho0U0sq).d;
}

double orc_timestep(void* h, const double* U, double cfl) {
  Solver* S = (Solver*)h;
  return S->timestep(U, cfl);
}

// Transposed residual Jacobian: out = (dR/dU)^T lam (reverse mode, exact).
int orc_rhs_vjp(void* h, const double* U, const double* lam, double* out, double t) {
  ((Solver*)h)->rhs_vjp(U, lam, out, t);
  return 0;
}

// Gradient of E_k at U (reverse mode).
int orc_kinetic_energy_grad(void* h, const double* U, double rho0U0sq, double* grad) {
  ((Solver*)h)->kinetic_energy_grad(U, rho0U0sq, grad);
  return 0;
}

// Reverse sweep of a whole trajectory: lamU <- (dU(T)/dU0)^T lamU.
int orc_lserk_adjoint(void* h, const double* U0, double* lamU, int nsteps, double dt, double t0) {
  if (nsteps < 0) { g_err = "negative step count"; return 1; }
  ((Solver*)h)->lserk_adjoint(U0, lamU, nsteps, dt, t0);
  return 0;
}

// Operation counts of one residual evaluation: {add/sub, mul, div, sqrt, log}.
int orc_rhs_opcount(void* h, const double* U, uint64_t* counts) {
  Solver* S = (Solver*)h;
  size_t n = (size_t)5 * S->nElems * S->n3;
  std::vector<orc::Cnt> X(n), Y(n);
  for (size_t i = 0; i < n; ++i) X[i] = orc::Cnt(U[i]);
  for (int e = 0; e < S->nElems; ++e) S->ensure_geom(e);
  for (int s = 0; s < S->nSides; ++s) S->ensure_side(s);
  orc::Cnt::n_add = orc::Cnt::n_mul = orc::Cnt::n_div = orc::Cnt::n_sqrt = orc::Cnt::n_log = 0;
  std::vector<int> all;
  S->rhs<orc::Cnt>(X.data(), Y.data(), 0.0, all);
  counts[0] = orc::Cnt::n_add; counts[1] = orc::Cnt::n_mul; counts[2] = orc::Cnt::n_div;
  counts[3] = orc::Cnt::n_sqrt; counts[4] = orc::Cnt::n_log;
  return 0;
}

// Point functions for unit pins.
void orc_flux_twopoint(const int* icfg, const double* dcfg, const double* Ua, const double* Ub, const double* nv,
                       double* F) {
  Solver S;
  S.C.twopoint = icfg[4]; S.C.gamma = dcfg[0];
  S.flux_twopoint<double>(Ua, Ub, nv, F);
}
void orc_flux_adv(const double* dcfg, const double* U, const double* nv, double* F) {
  Solver S; S.C.gamma = dcfg[0];
  S.flux_adv<double>(U, nv, F);
}
void orc_flux_visc(const double* dcfg, const double* U, const double* g, int n, double* G) {
  Solver S; S.C.gamma = dcfg[0]; S.C.mu = dcfg[1]; S.C.Pr = dcfg[2]; S.C.R = dcfg[3];
  S.flux_visc<double>(U, g, n, G);
}
void orc_flux_visc_law(const int* icfg, const double* dcfg, const double* U, const double* g, int n, double* G) {
  Solver S; S.C.gamma = dcfg[0]; S.C.mu = dcfg[1]; S.C.Pr = dcfg[2]; S.C.R = dcfg[3];
  S.C.viscosity = icfg[8]; S.C.Tref = dcfg[6]; S.C.Ts = dcfg[7];
  S.flux_visc<double>(U, g, n, G);
}
double orc_viscosity(const int* icfg, const double* dcfg, double temp) {
  Solver S; S.C.mu = dcfg[1]; S.C.viscosity = icfg[8]; S.C.Tref = dcfg[6]; S.C.Ts = dcfg[7];
  return S.viscosity<double>(temp);
}
void orc_roe_matrix(const double* dcfg, const double* UL, const double* UR, const double* nh, int mode, double* D) {
  Solver S; S.C.gamma = dcfg[0];
  S.roe_matrix<double>(UL, UR, nh, mode, D);
}
// FV sub-cells: element types (1 = FV), conversions, indicator, geometry, operators.
int orc_fv_set_mask(void* h, const int* mask) {
  Solver* S = (Solver*)h;
  if (!S->C.fv) { g_err = "FV sub-cells not enabled"; return 1; }
  for (int e = 0; e < S->nElems; ++e) S->fvmask[e] = mask[e] ? 1 : 0;
  return 0;
}
int orc_fv_switch(void* h, double* U, double* dU, const int* newmask) {
  Solver* S = (Solver*)h;
  if (!S->C.fv) { g_err = "FV sub-cells not enabled"; return 1; }
  S->fv_switch(U, dU, newmask);
  return 0;
}
void orc_fv_get_mask(void* h, int* mask) {
  Solver* S = (Solver*)h;
  for (int e = 0; e < S->nElems; ++e) mask[e] = S->C.fv ? S->fvmask[e] : 0;
}
int orc_fv_indicator(void* h, const double* U, double* ind) {
  Solver* S = (Solver*)h;
  for (int e = 0; e < S->nElems; ++e) { S->ensure_geom(e); ind[e] = S->indicator(U, e); }
  return 0;
}
// Sub-cell volumes [nElems][n3], interior sub-face vectors [nElems][3][3][N][n2],
// boundary sub-face vectors [nSides][3][n2].
int orc_fv_geometry(void* h, double* V, double* Si, double* Sb) {
  Solver* S = (Solver*)h;
  if (!S->C.fv) { g_err = "FV sub-cells not enabled"; return 1; }
  const size_t ni = (size_t)9 * S->C.N * S->n2;
  for (int e = 0; e < S->nElems; ++e) {
    S->ensure_fv_geom(e);
    for (int t = 0; t < S->n3; ++t) V[(size_t)e * S->n3 + t] = S->Vsub[e][t];
    for (size_t x = 0; x < ni; ++x) Si[(size_t)e * ni + x] = S->Sint[e][x];
  }
  for (int s = 0; s < S->nSides; ++s) {
    S->ensure_fv_side(s);
    for (int x = 0; x < 3 * S->n2; ++x) Sb[(size_t)s * 3 * S->n2 + x] = S->Sbnd[s][x];
  }
  return 0;
}
int orc_fv_operators(void* h, double* Bs, double* Bsi, double* Vli) {
  Solver* S = (Solver*)h;
  if (!S->C.fv) { g_err = "FV sub-cells not enabled"; return 1; }
  for (int x = 0; x < S->n1 * S->n1; ++x) { Bs[x] = S->Bsub[x]; Bsi[x] = S->Bsubinv[x]; Vli[x] = S->Vleginv[x]; }
  return 0;
}
// Sub-cell gradients of every element [12][nElems][n3] (Navier-Stokes FV
// contexts): Green-Gauss for FV elements, the sub-cell means of the lifted
// gradient for DG elements.
int orc_fv_gradients(void* h, const double* U, double* g) {
  Solver* S = (Solver*)h;
  if (!S->C.fv || S->C.physics != 1) { g_err = "FV gradients: Navier-Stokes FV contexts only"; return 1; }
  Solver::Work<double> W;
  W.tr.assign(S->nSides, {}); W.gtr.assign(S->nSides, {}); W.g.assign(S->nElems, {});
  S->ensure_fv_caches(W);
  for (int e = 0; e < S->nElems; ++e) {
    const std::vector<double>& G = S->elem_grad(U, e, W);
    for (int c = 0; c < 12; ++c)
      for (int t = 0; t < S->n3; ++t) g[((size_t)c * S->nElems + e) * S->n3 + t] = G[(size_t)c * S->n3 + t];
  }
  return 0;
}
// Element-wise DG -> FV (dir 0) or FV -> DG (dir 1) of a [5][n3] block.
int orc_fv_convert(void* h, int e, int dir, const double* in, double* out) {
  Solver* S = (Solver*)h;
  if (!S->C.fv || e < 0 || e >= S->nElems) { g_err = "bad FV conversion request"; return 1; }
  if (dir == 0) S->dg_to_fv(e, in, out); else S->fv_to_dg(e, in, out);
  return 0;
}

void orc_entropy_vars(const double* dcfg, const double* U, double* v) {
  Solver S; S.C.gamma = dcfg[0];
  S.entropy_vars<double>(U, v);
}
void orc_cons_from_entropy(const double* dcfg, const double* v, double* U) {
  Solver S; S.C.gamma = dcfg[0];
  S.cons_from_entropy<double>(v, U);
}
// Operation counts {add/sub, mul, div, sqrt, log} of one point function on
// the counting scalar: kind 0 flux_adv(Ua, nv), 1 logmean(Ua[0], Ub[0]),
// 2 flux_twopoint(Ua, Ub, nv) (Chandrashekar).
int orc_opcount_point(int kind, const double* dcfg, const double* Ua, const double* Ub, const double* nv,
                      uint64_t* counts) {
  Solver S;
  S.C.gamma = dcfg[0];
  orc::Cnt a[5], b[5], F[5];
  for (int v = 0; v < 5; ++v) { a[v] = orc::Cnt(Ua[v]); b[v] = orc::Cnt(Ub[v]); }
  orc::Cnt::n_add = orc::Cnt::n_mul = orc::Cnt::n_div = orc::Cnt::n_sqrt = orc::Cnt::n_log = 0;
  if (kind == 0) S.flux_adv<orc::Cnt>(a, nv, F);
  else if (kind == 1) F[0] = S.logmean<orc::Cnt>(a[0], b[0]);
  else if (kind == 2) S.flux_twopoint<orc::Cnt>(a, b, nv, F);
  else { g_err = "unknown point function"; return 1; }
  counts[0] = orc::Cnt::n_add; counts[1] = orc::Cnt::n_mul; counts[2] = orc::Cnt::n_div;
  counts[3] = orc::Cnt::n_sqrt; counts[4] = orc::Cnt::n_log;
  return 0;
}

double orc_logmean(double x, double y) {
  Solver S;
  return S.logmean<double>(x, y);
}
void orc_mms_source(const double* dcfg, double x, double y, double z, double t, double* Q) {
  Solver S; S.C.gamma = dcfg[0]; S.C.mu = dcfg[1]; S.C.Pr = dcfg[2]; S.C.R = dcfg[3];
  S.C.mms_A = dcfg[4]; S.C.mms_a = dcfg[5];
  S.mms_source(x, y, z, t, Q);
}

}  // extern "C"

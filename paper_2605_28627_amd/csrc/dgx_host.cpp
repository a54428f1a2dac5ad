// dgx_host.cpp -- host runtime and C-ABI of the DGSEM residual library.
//
// Host side of the library: validation of every ABI argument, the 1-D basis,
// the per-element face table, the metric terms (conservative curl form),
// device uploads, workspace planning and the launch sequence of the hot path.
// All arithmetic of the residual itself runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dgx.h"
#include "dgx_internal.hpp"

using namespace dgx;

struct dg_ctx {
  dg_config cfg{};
  Phys phys{};
  int N = 0, n1 = 0, n2 = 0, n3 = 0;
  // basis (host)
  std::vector<double> x, w, D, Lm, Lp;
  DevBasis hb{};
  // mesh (host)
  int nElems = 0, nSides = 0, Ngeo = 0;
  bool mesh_set = false, mesh_on_device = false;
  std::vector<int> efc;                 // [nElems*6]
  std::vector<double> xyz, Ja, sJ;      // [3][nE][n3], [9][nE][n3], [nE][n3]
  std::vector<double> nvec;             // [3][nSides][n2] master outward n*s
  std::vector<double> wJ;               // quadrature weight times J: [nE][n3]
  double volume = 0.0;
  // device (library-owned)
  double* d_Ja = nullptr;               // [10][nE][n3]: Ja, then 1/J (d_sJ = d_Ja + 9 nE n3)
  double* d_sJ = nullptr;
  double* d_em = nullptr;               // [10][nE]: constant metric terms per element (Geo::em)
  bool elem_metrics = true;             // kernels take constant elements' terms from d_em
  int n_const_metric = 0;               // elements with constant metric terms in d_em
  double* d_face = nullptr;
  int* d_efc = nullptr;
  DevBasis* d_basis = nullptr;
  // FV sub-cells (cfg.fv): geometry, element types, side flags
  std::vector<int> side_elem;           // [2*nSides] (host)
  double* d_fvV = nullptr;
  double* d_fvS = nullptr;
  double* d_fvSb = nullptr;
  int* d_etype = nullptr;
  int* d_etype_new = nullptr;
  int* d_sidefv = nullptr;
  int* d_efv = nullptr;
  int* d_side_elem = nullptr;
  // workspace (caller-owned)
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  // profiling: pairs of events per launch, grouped by kernel family
  bool prof = false;
  int prof_mask = 0;   // families bracketed by events (bit f = family f)
  struct Rec { int fam; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double prof_ms[6] = {0, 0, 0, 0, 0, 0};
  long prof_n[6] = {0, 0, 0, 0, 0, 0};
};

enum { FAM_TRACE = 0, FAM_LIFT = 1, FAM_VOLUME = 2, FAM_ADJOINT = 3, FAM_OTHER = 4, FAM_FV = 5 };
static const char* kFamNames[6] = {"trace", "lift", "volume", "adjoint", "other", "fv"};

static hipEvent_t pool_event(dg_ctx* c) {
  if (!c->pool.empty()) { hipEvent_t e = c->pool.back(); c->pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when profiling is on.
struct ProfScope {
  dg_ctx* c; int fam; hipStream_t s; hipEvent_t a = nullptr, b = nullptr;
  ProfScope(dg_ctx* c_, int fam_, hipStream_t s_) : c(c_), fam(fam_), s(s_) {
    if (c->prof && ((c->prof_mask >> fam) & 1)) { a = pool_event(c); b = pool_event(c); if (a) (void)hipEventRecord(a, s); }
  }
  ~ProfScope() {
    if (a && b) { (void)hipEventRecord(b, s); c->recs.push_back({fam, a, b}); }
  }
};

// Folds finished records into the totals (synchronises on the last event).
static void prof_collect(dg_ctx* c) {
  for (auto& r : c->recs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->prof_ms[r.fam] += ms;
      c->prof_n[r.fam] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
}

static thread_local std::string g_thread_err;

static dg_status fail(dg_ctx* c, dg_status st, const std::string& msg) {
  if (c) c->err = msg;
  g_thread_err = msg;
  return st;
}

#define HIPCHK(ctx, call)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(ctx, DG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// 1-D basis.  Gauss nodes are the zeros of P_{N+1}; Lobatto nodes are +-1 and
// the zeros of q = P_{N+1} - P_{N-1} in the interior (both by Newton on the
// three-term recurrence).  D_{al} = l_l'(x_a) from barycentric weights with
// the diagonal fixed so that D annihilates constants.
// ---------------------------------------------------------------------------
static void leg_eval(int n, double x, double* Pn, double* dPn, double* Pnm1, double* dPnm1) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { *Pn = 1.0; *dPn = 0.0; *Pnm1 = 0.0; *dPnm1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    double d2 = d0 + (2 * k - 1) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *Pn = p1; *dPn = d1; *Pnm1 = p0; *dPnm1 = d0;
}

static bool host_basis(int N, int nodes, std::vector<double>& x, std::vector<double>& w) {
  const int n1 = N + 1;
  const double pi = 3.14159265358979323846;
  x.assign(n1, 0.0); w.assign(n1, 0.0);
  if (nodes == DG_NODES_GAUSS) {
    for (int j = 0; j <= N / 2; ++j) {
      double z = -std::cos((2 * j + 1) * pi / (2 * N + 2));
      for (int it = 0; it < 200; ++it) {
        double P, dP, Pm, dPm;
        leg_eval(N + 1, z, &P, &dP, &Pm, &dPm);
        double dz = P / dP;
        z -= dz;
        if (std::fabs(dz) < 4e-17 * std::fabs(z) + 1e-300) break;
      }
      double P, dP, Pm, dPm;
      leg_eval(N + 1, z, &P, &dP, &Pm, &dPm);
      x[j] = z; x[N - j] = -z;
      w[j] = w[N - j] = 2.0 / ((1.0 - z * z) * dP * dP);
    }
  } else {
    x[0] = -1.0; x[N] = 1.0;
    for (int j = 1; j <= (N - 1) / 2; ++j) {
      double z = -std::cos((j + 0.25) * pi / N - 3.0 / (8.0 * N * pi * (j + 0.25)));
      for (int it = 0; it < 200; ++it) {
        // q = P_{N+1} - P_{N-1}, q' = P'_{N+1} - P'_{N-1}
        double Pa, dPa, Pb, dPb, Pc, dPc, Pd, dPd;
        leg_eval(N + 1, z, &Pa, &dPa, &Pb, &dPb);   // P_{N+1}, P_N
        leg_eval(N - 1, z, &Pc, &dPc, &Pd, &dPd);   // P_{N-1}
        double q = Pa - Pc, dq = dPa - dPc;
        double dz = q / dq;
        z -= dz;
        if (std::fabs(dz) < 4e-17 * std::fabs(z) + 1e-300) break;
      }
      x[j] = z; x[N - j] = -z;
    }
    if (N % 2 == 0) x[N / 2] = 0.0;
    for (int j = 0; j < n1; ++j) {
      double P, dP, Pm, dPm;
      leg_eval(N, x[j], &P, &dP, &Pm, &dPm);
      w[j] = 2.0 / (N * (N + 1.0) * P * P);
    }
  }
  if (nodes == DG_NODES_GAUSS && (N % 2 == 0)) x[N / 2] = 0.0;
  return true;
}

static void host_diff(const std::vector<double>& x, std::vector<double>& D) {
  const int n = (int)x.size();
  std::vector<double> bw(n);
  for (int j = 0; j < n; ++j) {
    double p = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) p *= (x[j] - x[k]);
    bw[j] = 1.0 / p;
  }
  D.assign(n * n, 0.0);
  for (int a = 0; a < n; ++a) {
    double rs = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == a) continue;
      double v = bw[l] / bw[a] / (x[a] - x[l]);
      D[a * n + l] = v;
      rs += v;
    }
    D[a * n + a] = -rs;
  }
}

static double lagrange_at(const std::vector<double>& nodes, int j, double z) {
  double v = 1.0;
  for (int k = 0; k < (int)nodes.size(); ++k)
    if (k != j) v *= (z - nodes[k]) / (nodes[j] - nodes[k]);
  return v;
}

// Apply a 1-D operator M (rows x cols, row-major) along dimension dim of a
// [n_k][n_j][n_i] array; the operated dimension changes size from cols to rows.
static void apply_dim(const double* M, int rows, int cols, const double* in, int ni, int nj, int nk, int dim,
                      double* out) {
  int oi = ni, oj = nj, ok = nk;
  if (dim == 0) oi = rows; else if (dim == 1) oj = rows; else ok = rows;
  for (int k = 0; k < ok; ++k)
    for (int j = 0; j < oj; ++j)
      for (int i = 0; i < oi; ++i) {
        double s = 0.0;
        for (int m = 0; m < cols; ++m) {
          int ii = i, jj = j, kk = k;
          int r = (dim == 0) ? i : (dim == 1) ? j : k;
          if (dim == 0) ii = m; else if (dim == 1) jj = m; else kk = m;
          s += M[r * cols + m] * in[((size_t)kk * nj + jj) * ni + ii];
        }
        out[((size_t)k * oj + j) * oi + i] = s;
      }
}

// Host threads for element-parallel set-up work: up to the hardware's count
// (at most 16), and at least `grain` elements per thread.
static int host_threads(int nitems, int grain) {
  int hw = (int)std::thread::hardware_concurrency();
  if (hw < 1) hw = 1;
  if (hw > 16) hw = 16;
  int n = nitems / grain;
  return n < 1 ? 1 : (n < hw ? n : hw);
}

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
extern "C" {

const char* dg_last_error(const dg_ctx* ctx) { return ctx ? ctx->err.c_str() : g_thread_err.c_str(); }

dg_status dg_lserk_coefficients(double* A5, double* B5, double* c5) {
  if (!A5 || !B5 || !c5) return fail(nullptr, DG_ERR_ARG, "null pointer");
  // Carpenter & Kennedy (1994), five-stage fourth-order 2N-storage scheme.
  const double A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                       -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
  const double B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                       1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                       2277821191437.0 / 14882151754819.0};
  const double C[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                       2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};
  for (int s = 0; s < 5; ++s) { A5[s] = A[s]; B5[s] = B[s]; c5[s] = C[s]; }
  return DG_OK;
}

// Niegemann, Diehl & Busch (2012), fourteen-stage fourth-order 2N-storage
// scheme (their RK4-14 coefficients).
static const double kRK14A[14] = {0.0, -0.7188012108672410, -0.7785331173421570, -0.0053282796654044,
                                  -0.8552979934029281, -3.9564138245774565, -1.5780575380587385,
                                  -2.0837094552574054, -0.7483334182761610, -0.7032861106563359,
                                  0.0013917096117681, -0.0932075369637460, -0.9514200470875948,
                                  -7.1151571693922548};
static const double kRK14B[14] = {0.0367762454319673, 0.3136296607553959, 0.1531848691869027, 0.0030097086818182,
                                  0.3326293790646110, 0.2440251405350864, 0.3718879239592277,
                                  0.6204126221582444, 0.1524043173028741, 0.0760894927419266,
                                  0.0077604214040978, 0.0024647284755382, 0.0780348340049386,
                                  5.5059777270269628};
static const double kRK14C[14] = {0.0, 0.0367762454319673, 0.1249685262725025, 0.2446177702277698,
                                  0.2476149531070420, 0.2969311120382472, 0.3978149645802642,
                                  0.5270854589440328, 0.6981269994175695, 0.8190890835352128,
                                  0.8527059887098624, 0.8604711817462826, 0.8627060376969976,
                                  0.8734213127600976};

dg_status dg_rk_coefficients(int integrator, double* A, double* B, double* c, int* nstages) {
  if (!A || !B || !c || !nstages) return fail(nullptr, DG_ERR_ARG, "dg_rk_coefficients: null pointer");
  if (integrator == DG_RK_LSERK45) {
    *nstages = 5;
    return dg_lserk_coefficients(A, B, c);
  }
  if (integrator == DG_RK_LSERK414) {
    *nstages = 14;
    for (int s = 0; s < 14; ++s) { A[s] = kRK14A[s]; B[s] = kRK14B[s]; c[s] = kRK14C[s]; }
    return DG_OK;
  }
  return fail(nullptr, DG_ERR_ARG, "dg_rk_coefficients: unknown integrator");
}

// ---------------------------------------------------------------------------
// FV sub-cell operators: Bs[k][i] = integral of l_i over the k-th of the N+1
// equal sub-intervals of [-1,1] (Gauss rule with N+1 points, exact for the
// degree-N integrand), its inverse, and the inverse of the Vandermonde of the
// orthonormal Legendre polynomials sqrt((2m+1)/2) P_m at the nodes.
// ---------------------------------------------------------------------------
static bool invert_small(std::vector<double> A, int n, double* inv) {
  std::vector<double> I((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)piv * n + c])) piv = r;
    if (A[(size_t)piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) { std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]); std::swap(I[(size_t)c * n + k], I[(size_t)piv * n + k]); }
    const double d = 1.0 / A[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) { A[(size_t)c * n + k] *= d; I[(size_t)c * n + k] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { A[(size_t)r * n + k] -= f * A[(size_t)c * n + k]; I[(size_t)r * n + k] -= f * I[(size_t)c * n + k]; }
    }
  }
  std::copy(I.begin(), I.end(), inv);
  return true;
}

static void fv_operators(int n1, const std::vector<double>& x, DevBasis& b) {
  std::vector<double> xg, wg;
  host_basis(n1 - 1, DG_NODES_GAUSS, xg, wg);
  std::vector<double> Bs((size_t)n1 * n1), V((size_t)n1 * n1);
  for (int k = 0; k < n1; ++k) {
    const double lo = -1.0 + 2.0 * k / n1, h = 2.0 / n1;
    for (int i = 0; i < n1; ++i) {
      double s = 0.0;
      for (int g = 0; g < n1; ++g) s += wg[g] * lagrange_at(x, i, lo + 0.5 * h * (xg[g] + 1.0));
      Bs[(size_t)k * n1 + i] = 0.5 * h * s;
    }
  }
  for (int i = 0; i < n1; ++i)
    for (int m = 0; m < n1; ++m) {
      double P, dP, Pm, dPm;
      leg_eval(m, x[i], &P, &dP, &Pm, &dPm);
      V[(size_t)i * n1 + m] = std::sqrt((2.0 * m + 1.0) / 2.0) * P;
    }
  for (int t = 0; t < n1 * n1; ++t) b.Bs[t] = Bs[t];
  invert_small(Bs, n1, b.Bsi);
  invert_small(V, n1, b.Vli);
}

dg_status dg_create(const dg_config* cfg, dg_ctx** out) {
  if (!cfg || !out) return fail(nullptr, DG_ERR_ARG, "dg_create: null pointer");
  *out = nullptr;
  const dg_config& c = *cfg;
  if (c.nodes != DG_NODES_GAUSS && c.nodes != DG_NODES_LOBATTO) return fail(nullptr, DG_ERR_ARG, "dg_create: nodes");
  if (c.volume_form != DG_FORM_WEAK && c.volume_form != DG_FORM_SPLIT) return fail(nullptr, DG_ERR_ARG, "dg_create: volume_form");
  if (c.physics != DG_PHYS_EULER && c.physics != DG_PHYS_NAVIER_STOKES) return fail(nullptr, DG_ERR_ARG, "dg_create: physics");
  if (c.riemann != DG_RIEMANN_RUSANOV && c.riemann != DG_RIEMANN_CENTRAL && c.riemann != DG_RIEMANN_ROE)
    return fail(nullptr, DG_ERR_ARG, "dg_create: riemann");
  if (c.viscosity != DG_VISC_CONSTANT && c.viscosity != DG_VISC_SUTHERLAND) return fail(nullptr, DG_ERR_ARG, "dg_create: viscosity");
  if (c.viscosity == DG_VISC_SUTHERLAND && (!(c.Tref > 0.0) || !(c.Ts >= 0.0) || !std::isfinite(c.Tref) || !std::isfinite(c.Ts)))
    return fail(nullptr, DG_ERR_ARG, "dg_create: Sutherland constants");
  if (c.twopoint != DG_TWOPOINT_CHANDRASHEKAR && c.twopoint != DG_TWOPOINT_CENTRAL) return fail(nullptr, DG_ERR_ARG, "dg_create: twopoint");
  if (c.precision != DG_PREC_FP64 && c.precision != DG_PREC_FP32_FLUX) return fail(nullptr, DG_ERR_ARG, "dg_create: precision");
  if (c.integrator != DG_RK_LSERK45 && c.integrator != DG_RK_LSERK414) return fail(nullptr, DG_ERR_ARG, "dg_create: integrator");
  if (!(c.gamma > 1.0) || !(c.mu >= 0.0) || !(c.Pr > 0.0) || !(c.R > 0.0) || !std::isfinite(c.gamma) ||
      !std::isfinite(c.mu) || !std::isfinite(c.Pr) || !std::isfinite(c.R))
    return fail(nullptr, DG_ERR_ARG, "dg_create: gas constants");
  if (c.N < 1 || c.N > kMaxN) return fail(nullptr, DG_ERR_UNSUPPORTED, "dg_create: N must be in 1..7");
  if (c.fv != 0 && c.fv != 1) return fail(nullptr, DG_ERR_ARG, "dg_create: fv");
  if (c.fv && (c.precision != DG_PREC_FP64 || c.riemann != DG_RIEMANN_RUSANOV ||
               (c.physics == DG_PHYS_NAVIER_STOKES && c.viscosity != DG_VISC_CONSTANT)))
    return fail(nullptr, DG_ERR_UNSUPPORTED,
                "dg_create: FV sub-cells cover FP64 and Rusanov (Navier-Stokes: constant viscosity)");
  dg_ctx* x = new (std::nothrow) dg_ctx();
  if (!x) return fail(nullptr, DG_ERR_NOMEM, "dg_create: host allocation");
  x->cfg = c;
  x->N = c.N; x->n1 = c.N + 1; x->n2 = x->n1 * x->n1; x->n3 = x->n2 * x->n1;
  x->phys.gamma = c.gamma; x->phys.gm1 = c.gamma - 1.0; x->phys.igm1 = 1.0 / (c.gamma - 1.0); x->phys.mu = c.mu;
  x->phys.lam = c.mu * c.gamma * c.R / ((c.gamma - 1.0) * c.Pr);
  x->phys.R = c.R; x->phys.Rinv = 1.0 / c.R; x->phys.Pr = c.Pr;
  x->phys.riemann = c.riemann; x->phys.twopoint = c.twopoint;
  x->phys.kappa = c.gamma * c.R / ((c.gamma - 1.0) * c.Pr);
  x->phys.visc_law = c.viscosity; x->phys.Tref = c.Tref; x->phys.Ts = c.Ts;
  host_basis(c.N, c.nodes, x->x, x->w);
  host_diff(x->x, x->D);
  const int n1 = x->n1;
  x->Lm.resize(n1); x->Lp.resize(n1);
  for (int j = 0; j < n1; ++j) { x->Lm[j] = lagrange_at(x->x, j, -1.0); x->Lp[j] = lagrange_at(x->x, j, 1.0); }
  DevBasis& b = x->hb;
  std::memset(&b, 0, sizeof(b));
  for (int a = 0; a < n1; ++a) {
    b.w[a] = x->w[a]; b.winv[a] = 1.0 / x->w[a]; b.Lm[a] = x->Lm[a]; b.Lp[a] = x->Lp[a];
    for (int l = 0; l < n1; ++l) {
      b.D[a * n1 + l] = x->D[a * n1 + l];
      b.Dhat[a * n1 + l] = x->w[l] / x->w[a] * x->D[l * n1 + a];
      // M^-1 (Q - Q^T) by the SBP property Q + Q^T = Lp Lp^T - Lm Lm^T (exactly
      // 2D with the two corner terms on LGL nodes, where Lm = e_0, Lp = e_N)
      b.DS[a * n1 + l] = 2.0 * x->D[a * n1 + l] - (x->Lp[a] * x->Lp[l] - x->Lm[a] * x->Lm[l]) / x->w[a];
    }
  }
  if (c.fv) fv_operators(n1, x->x, b);
  *out = x;
  return DG_OK;
}

static void free_events(dg_ctx* c) {
  for (auto& r : c->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  c->recs.clear();
  for (auto e : c->pool) (void)hipEventDestroy(e);
  c->pool.clear();
}

static void free_device(dg_ctx* c) {
  if (c->d_Ja) (void)hipFree(c->d_Ja);   // (d_sJ lies in the same allocation)
  if (c->d_em) (void)hipFree(c->d_em);
  if (c->d_face) (void)hipFree(c->d_face);
  if (c->d_efc) (void)hipFree(c->d_efc);
  if (c->d_basis) (void)hipFree(c->d_basis);
  for (double** p : {&c->d_fvV, &c->d_fvS, &c->d_fvSb})
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  for (int** p : {&c->d_etype, &c->d_etype_new, &c->d_sidefv, &c->d_efv, &c->d_side_elem})
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  c->d_Ja = c->d_sJ = c->d_em = c->d_face = nullptr;
  c->n_const_metric = 0;
  c->d_efc = nullptr;
  c->d_basis = nullptr;
  c->mesh_on_device = false;
}

dg_status dg_destroy(dg_ctx* ctx) {
  if (!ctx) return DG_OK;
  free_events(ctx);
  free_device(ctx);
  delete ctx;
  return DG_OK;
}

dg_status dg_set_reference_state(dg_ctx* c, double rho0, double p0) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_set_reference_state: null context");
  if (rho0 == 0.0 && p0 == 0.0) {
    c->phys.p0 = c->phys.ib0 = c->phys.h0 = 0.0;
    return DG_OK;
  }
  if (!(rho0 > 0.0) || !(p0 > 0.0) || !std::isfinite(rho0) || !std::isfinite(p0))
    return fail(c, DG_ERR_ARG, "dg_set_reference_state: need rho0 > 0 and p0 > 0 (or both 0)");
  c->phys.p0 = p0;
  c->phys.ib0 = 2.0 * p0 / rho0;
  c->phys.h0 = c->cfg.gamma * p0 / (c->cfg.gamma - 1.0);
  return DG_OK;
}

// ---------------------------------------------------------------------------
// Mesh and metrics
// ---------------------------------------------------------------------------
// An affine element (x = x0 + A xi) has constant metric terms, Ja = cof(A)
// and J = det(A); computed node by node they still differ in the last bits
// (the curl form sums D-weighted products).  When every one of the nine
// components and 1/J stays within 1e-12 of its largest magnitude over the
// element's nodes, every node is given the element's mean instead: the
// terms then are exactly constant, which the kernels recognise (elem_metrics).
// Ja points at component 0 of the element (components stride cs), sJ at its 1/J.
static void snap_affine(double* Ja, size_t cs, double* sJ, int n3) {
  double mean[10];
  for (int c = 0; c < 10; ++c) {
    const double* v = c < 9 ? Ja + c * cs : sJ;
    double s = 0.0;
    for (int t = 0; t < n3; ++t) s += v[t];
    mean[c] = s / n3;
  }
  double scale = 0.0;   // largest metric entry of the element
  for (int c = 0; c < 9; ++c)
    for (int t = 0; t < n3; ++t) scale = std::max(scale, std::fabs(Ja[c * cs + t]));
  for (int c = 0; c < 10; ++c) {
    const double* v = c < 9 ? Ja + c * cs : sJ;
    const double tol = 1e-12 * (c < 9 ? scale : std::fabs(mean[9]));
    for (int t = 0; t < n3; ++t)
      if (!(std::fabs(v[t] - mean[c]) <= tol)) return;
  }
  for (int c = 0; c < 10; ++c) {
    double* v = c < 9 ? Ja + c * cs : sJ;
    for (int t = 0; t < n3; ++t) v[t] = mean[c];
  }
}

// The per-element copy of the metric terms (Geo::em, [10][nE]: Ja^r_n at
// 3r+n, 1/J at 9) for every element whose terms are bitwise the same at all
// of its nodes; 1/J = 0 marks the others, whose kernels read the node arrays.
static dg_status upload_elem_metrics(dg_ctx* c) {
  const size_t nE = c->nElems, n3 = c->n3;
  if (!c->d_em) {
    hipError_t e = hipMalloc((void**)&c->d_em, 10 * nE * sizeof(double));
    if (e != hipSuccess)
      return fail(c, e == hipErrorOutOfMemory ? DG_ERR_NOMEM : DG_ERR_HIP,
                  std::string("element metrics: hipMalloc: ") + hipGetErrorString(e));
  }
  std::vector<double> em(10 * nE, 0.0);
  int count = 0;
  for (size_t e = 0; e < nE && c->elem_metrics; ++e) {
    bool same = true;
    for (int comp = 0; comp < 10 && same; ++comp) {
      const double* v = comp < 9 ? &c->Ja[(comp * nE + e) * n3] : &c->sJ[e * n3];
      for (size_t t = 1; t < n3 && same; ++t) same = v[t] == v[0];
    }
    if (!same) continue;
    for (int comp = 0; comp < 9; ++comp) em[comp * nE + e] = c->Ja[(comp * nE + e) * n3];
    em[9 * nE + e] = c->sJ[e * n3];
    ++count;
  }
  HIPCHK(c, hipMemcpy(c->d_em, em.data(), em.size() * sizeof(double), hipMemcpyHostToDevice));
  c->n_const_metric = count;
  return DG_OK;
}

dg_status dg_set_mesh(dg_ctx* c, int nElems, int Ngeo, const double* X, int nSides, const int* side_elem,
                      const int* side_loc, const int* side_orient) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_set_mesh: null context");
  if (!X || !side_elem || !side_loc || !side_orient) return fail(c, DG_ERR_ARG, "dg_set_mesh: null pointer");
  if (nElems <= 0 || Ngeo < 1 || Ngeo > 16 || nSides <= 0) return fail(c, DG_ERR_ARG, "dg_set_mesh: sizes");
  if ((long long)nSides * 2 != (long long)nElems * 6)
    return fail(c, DG_ERR_MESH, "dg_set_mesh: a closed conforming hexahedral mesh has 3 sides per element");
  if ((long long)nSides >= (1LL << 27)) return fail(c, DG_ERR_UNSUPPORTED, "dg_set_mesh: too many sides");
  const int N = c->N, n1 = c->n1, n2 = c->n2, n3 = c->n3, g1 = Ngeo + 1;
  c->mesh_set = false;
  // face table
  std::vector<int> efc((size_t)nElems * 6, -1);
  for (int s = 0; s < nSides; ++s) {
    int o = side_orient[s];
    if (o < 0 || o > 7) return fail(c, DG_ERR_MESH, "dg_set_mesh: orientation out of range");
    for (int m = 0; m < 2; ++m) {
      int e = side_elem[2 * s + m], f = side_loc[2 * s + m];
      if (e < 0 || e >= nElems || f < 0 || f > 5) return fail(c, DG_ERR_MESH, "dg_set_mesh: side entry out of range");
      int& slotref = efc[(size_t)e * 6 + f];
      if (slotref != -1) return fail(c, DG_ERR_MESH, "dg_set_mesh: element face used twice");
      slotref = efc_pack(s, m, m == 0 ? 0 : o);
    }
  }
  for (size_t t = 0; t < efc.size(); ++t)
    if (efc[t] < 0) return fail(c, DG_ERR_MESH, "dg_set_mesh: element face without a side");
  // geometry: equispaced nodes -> solution nodes (relative to the element's
  // first geometry node; the metric terms are translation invariant)
  std::vector<double> xg(g1);
  for (int m = 0; m < g1; ++m) xg[m] = -1.0 + 2.0 * m / Ngeo;
  std::vector<double> V((size_t)n1 * g1);
  for (int a = 0; a < n1; ++a)
    for (int m = 0; m < g1; ++m) V[(size_t)a * g1 + m] = lagrange_at(xg, m, c->x[a]);
  std::vector<double> xyz((size_t)3 * nElems * n3), Ja((size_t)9 * nElems * n3), sJ((size_t)nElems * n3);
  // Elements are independent: a contiguous block of elements per host thread,
  // each with its own scratch.  The first element (in index order) with a
  // non-positive Jacobian is reported, whatever the thread count.
  auto elem_block = [&](int e0, int e1, int* bad_elem, double* bad_J) {
    std::vector<double> t1((size_t)g1 * g1 * n1), t2((size_t)g1 * n1 * n1), Xe((size_t)3 * n3), dX((size_t)9 * n3),
        prod((size_t)n3), dprod((size_t)n3), acc((size_t)n3), rel((size_t)g1 * g1 * g1);
    for (int e = e0; e < e1; ++e) {
      for (int d = 0; d < 3; ++d) {
        const double* src = X + ((size_t)d * nElems + e) * g1 * g1 * g1;
        const double x0 = src[0];
        for (int t = 0; t < g1 * g1 * g1; ++t) rel[t] = src[t] - x0;
        apply_dim(V.data(), n1, g1, rel.data(), g1, g1, g1, 0, t1.data());
        apply_dim(V.data(), n1, g1, t1.data(), n1, g1, g1, 1, t2.data());
        apply_dim(V.data(), n1, g1, t2.data(), n1, n1, g1, 2, &Xe[(size_t)d * n3]);
        for (int r = 0; r < 3; ++r) apply_dim(c->D.data(), n1, n1, &Xe[(size_t)d * n3], n1, n1, n1, r, &dX[(size_t)(3 * d + r) * n3]);
        for (int t = 0; t < n3; ++t) xyz[((size_t)d * nElems + e) * n3 + t] = Xe[(size_t)d * n3 + t] + x0;
      }
      for (int t = 0; t < n3; ++t) {
        double a[3][3];
        for (int d = 0; d < 3; ++d)
          for (int r = 0; r < 3; ++r) a[d][r] = dX[(size_t)(3 * d + r) * n3 + t];
        double J = a[0][0] * (a[1][1] * a[2][2] - a[2][1] * a[1][2]) + a[1][0] * (a[2][1] * a[0][2] - a[0][1] * a[2][2]) +
                   a[2][0] * (a[0][1] * a[1][2] - a[1][1] * a[0][2]);
        if (!(J > 0.0)) {
          *bad_elem = e;
          *bad_J = J;
          return;
        }
        sJ[(size_t)e * n3 + t] = 1.0 / J;
      }
      // Conservative curl form: Ja^r_n = -[curl_xi (X_l grad_xi X_m)]_r with
      // (n, m, l) cyclic; the product is collocated at the solution nodes.
      for (int n = 0; n < 3; ++n) {
        const int m = (n + 1) % 3, l = (n + 2) % 3;
        for (int r = 0; r < 3; ++r) {
          const int r1 = (r + 1) % 3, r2 = (r + 2) % 3;
          // Ja^r_n = d_{r2}(X_l d_{r1} X_m) - d_{r1}(X_l d_{r2} X_m)
          for (int t = 0; t < n3; ++t) prod[t] = Xe[(size_t)l * n3 + t] * dX[(size_t)(3 * m + r1) * n3 + t];
          apply_dim(c->D.data(), n1, n1, prod.data(), n1, n1, n1, r2, acc.data());
          for (int t = 0; t < n3; ++t) prod[t] = Xe[(size_t)l * n3 + t] * dX[(size_t)(3 * m + r2) * n3 + t];
          apply_dim(c->D.data(), n1, n1, prod.data(), n1, n1, n1, r1, dprod.data());
          for (int t = 0; t < n3; ++t) Ja[((size_t)(3 * r + n) * nElems + e) * n3 + t] = acc[t] - dprod[t];
        }
      }
      snap_affine(&Ja[(size_t)e * n3], (size_t)nElems * n3, &sJ[(size_t)e * n3], n3);
    }
  };
  {
    const int nth = host_threads(nElems, 64);
    std::vector<int> bad_elem(nth, -1);
    std::vector<double> bad_J(nth, 0.0);
    std::vector<std::thread> pool;
    for (int th = 0; th < nth; ++th) {
      const int e0 = (int)((long long)nElems * th / nth), e1 = (int)((long long)nElems * (th + 1) / nth);
      pool.emplace_back(elem_block, e0, e1, &bad_elem[th], &bad_J[th]);
    }
    for (auto& th : pool) th.join();
    for (int th = 0; th < nth; ++th)
      if (bad_elem[th] >= 0) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "dg_set_mesh: non-positive Jacobian %g in element %d", bad_J[th], bad_elem[th]);
        return fail(c, DG_ERR_MESH, buf);
      }
  }
  // master face normals from the volume metrics (extrapolated along the normal line)
  std::vector<double> nvec((size_t)3 * nSides * n2);
  auto side_block = [&](int s0, int s1) {
    for (int s = s0; s < s1; ++s) {
      const int e = side_elem[2 * s], f = side_loc[2 * s], dir = f / 2;
      const double sg = (f & 1) ? 1.0 : -1.0;
      const std::vector<double>& L = (f & 1) ? c->Lp : c->Lm;
      for (int q = 0; q < n1; ++q)
        for (int p = 0; p < n1; ++p)
          for (int comp = 0; comp < 3; ++comp) {
            double v = 0.0;
            for (int a = 0; a < n1; ++a) {
              int i, j, k;
              if (dir == 0) { i = a; j = p; k = q; } else if (dir == 1) { i = p; j = a; k = q; } else { i = p; j = q; k = a; }
              v += L[a] * Ja[((size_t)(3 * dir + comp) * nElems + e) * n3 + (k * n1 + j) * n1 + i];
            }
            nvec[((size_t)comp * nSides + s) * n2 + q * n1 + p] = sg * v;
          }
    }
  };
  // quadrature weights w_i w_j w_k J per node, and each element's volume
  std::vector<double> wJ((size_t)nElems * n3), evol((size_t)nElems);
  auto wj_block = [&](int e0, int e1) {
    for (int e = e0; e < e1; ++e) {
      double ve = 0.0;
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            size_t t = (size_t)e * n3 + (k * n1 + j) * n1 + i;
            wJ[t] = c->w[i] * c->w[j] * c->w[k] / sJ[t];
            ve += wJ[t];
          }
      evol[e] = ve;
    }
  };
  {
    const int nth = host_threads(nElems, 64);
    std::vector<std::thread> pool;
    for (int th = 0; th < nth; ++th) {
      const int s0 = (int)((long long)nSides * th / nth), s1 = (int)((long long)nSides * (th + 1) / nth);
      const int e0 = (int)((long long)nElems * th / nth), e1 = (int)((long long)nElems * (th + 1) / nth);
      pool.emplace_back([&, s0, s1, e0, e1]() { side_block(s0, s1); wj_block(e0, e1); });
    }
    for (auto& th : pool) th.join();
  }
  // |Omega|, summed element by element in index order (independent of the thread count)
  double vol = 0.0;
  for (int e = 0; e < nElems; ++e) vol += evol[e];
  (void)N;
  c->nElems = nElems; c->nSides = nSides; c->Ngeo = Ngeo;
  c->efc.swap(efc); c->xyz.swap(xyz); c->Ja.swap(Ja); c->sJ.swap(sJ); c->nvec.swap(nvec); c->wJ.swap(wJ);
  c->side_elem.assign(side_elem, side_elem + 2 * (size_t)nSides);
  c->volume = vol;
  c->mesh_set = true;
  c->ws = nullptr; c->ws_bytes = 0;
  return DG_OK;
}

static dg_status upload_face(dg_ctx* c, const std::vector<double>& nvec) {
  const size_t nf = (size_t)c->nSides * c->n2;
  std::vector<double> face(4 * nf);
  for (size_t t = 0; t < nf; ++t) {
    double a = nvec[t], b = nvec[nf + t], d = nvec[2 * nf + t];
    double s = std::sqrt(a * a + b * b + d * d);
    if (!(s > 0.0)) return fail(c, DG_ERR_MESH, "zero face normal");
    face[t] = a / s; face[nf + t] = b / s; face[2 * nf + t] = d / s; face[3 * nf + t] = s;
  }
  HIPCHK(c, hipMemcpy(c->d_face, face.data(), face.size() * sizeof(double), hipMemcpyHostToDevice));
  return DG_OK;
}

// FV sub-cell geometry from the current metrics: volumes V = B3 J, interior
// sub-face vectors (Ja^r interpolated to the sub-cell planes, integrated over
// each sub-face) and element-face sub-face vectors (the master's n s
// integrated over each sub-face).
static dg_status build_fv(dg_ctx* c) {
  const int N = c->N, n1 = c->n1, n2 = c->n2, n3 = c->n3, nE = c->nElems, nS = c->nSides;
  const double* Bs = c->hb.Bs;
  std::vector<double> V((size_t)nE * n3), S((size_t)9 * nE * N * n2), Sb((size_t)3 * nS * n2);
  std::vector<double> J((size_t)n3), t1((size_t)n3), t2((size_t)n3);
  std::vector<double> Bm((size_t)n1 * n1);
  for (int t = 0; t < n1 * n1; ++t) Bm[t] = Bs[t];
  std::vector<double> lp((size_t)n1), pl((size_t)n2);
  for (int e = 0; e < nE; ++e) {
    for (int t = 0; t < n3; ++t) J[t] = 1.0 / c->sJ[(size_t)e * n3 + t];
    apply_dim(Bm.data(), n1, n1, J.data(), n1, n1, n1, 0, t1.data());
    apply_dim(Bm.data(), n1, n1, t1.data(), n1, n1, n1, 1, t2.data());
    apply_dim(Bm.data(), n1, n1, t2.data(), n1, n1, n1, 2, &V[(size_t)e * n3]);
    for (int r = 0; r < 3; ++r)
      for (int a = 0; a < N; ++a) {
        const double xp = -1.0 + 2.0 * (a + 1) / n1;
        for (int l = 0; l < n1; ++l) lp[l] = lagrange_at(c->x, l, xp);
        for (int comp = 0; comp < 3; ++comp) {
          const double* Jr = &c->Ja[((size_t)(3 * r + comp) * nE + e) * n3];
          for (int q = 0; q < n1; ++q)
            for (int p = 0; p < n1; ++p) {
              double v = 0.0;
              for (int l = 0; l < n1; ++l) {
                const int i = r == 0 ? l : p, j = r == 0 ? p : (r == 1 ? l : q), k = r == 2 ? l : q;
                v += lp[l] * Jr[(k * n1 + j) * n1 + i];
              }
              pl[q * n1 + p] = v;
            }
          for (int q = 0; q < n1; ++q)
            for (int p = 0; p < n1; ++p) {
              double v = 0.0;
              for (int b2 = 0; b2 < n1; ++b2)
                for (int a2 = 0; a2 < n1; ++a2) v += Bs[p * n1 + a2] * Bs[q * n1 + b2] * pl[b2 * n1 + a2];
              S[(((size_t)(3 * r + comp) * nE + e) * N + a) * n2 + q * n1 + p] = v;
            }
        }
      }
  }
  for (int comp = 0; comp < 3; ++comp)
    for (int s = 0; s < nS; ++s)
      for (int q = 0; q < n1; ++q)
        for (int p = 0; p < n1; ++p) {
          double v = 0.0;
          for (int b2 = 0; b2 < n1; ++b2)
            for (int a2 = 0; a2 < n1; ++a2)
              v += Bs[p * n1 + a2] * Bs[q * n1 + b2] * c->nvec[((size_t)comp * nS + s) * n2 + b2 * n1 + a2];
          Sb[((size_t)comp * nS + s) * n2 + q * n1 + p] = v;
        }
  HIPCHK(c, hipMemcpy(c->d_fvV, V.data(), V.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_fvS, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_fvSb, Sb.data(), Sb.size() * sizeof(double), hipMemcpyHostToDevice));
  return DG_OK;
}

dg_status dg_upload_mesh(dg_ctx* c, int nElems, int Ngeo, const double* X, int nSides, const int* side_elem,
                         const int* side_loc, const int* side_orient) {
  dg_status st = dg_set_mesh(c, nElems, Ngeo, X, nSides, side_elem, side_loc, side_orient);
  if (st != DG_OK) return st;
  free_device(c);
  const size_t nv = (size_t)c->nElems * c->n3, nf = (size_t)c->nSides * c->n2;
  hipError_t e;
  if ((e = hipMalloc((void**)&c->d_Ja, 10 * nv * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&c->d_face, 4 * nf * sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void**)&c->d_efc, (size_t)c->nElems * 6 * sizeof(int))) != hipSuccess ||
      (e = hipMalloc((void**)&c->d_basis, sizeof(DevBasis))) != hipSuccess) {
    free_device(c);
    return fail(c, e == hipErrorOutOfMemory ? DG_ERR_NOMEM : DG_ERR_HIP,
                std::string("dg_upload_mesh: hipMalloc: ") + hipGetErrorString(e));
  }
  c->d_sJ = c->d_Ja + 9 * nv;
  HIPCHK(c, hipMemcpy(c->d_Ja, c->Ja.data(), 9 * nv * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_sJ, c->sJ.data(), nv * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_efc, c->efc.data(), (size_t)c->nElems * 6 * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_basis, &c->hb, sizeof(DevBasis), hipMemcpyHostToDevice));
  st = upload_face(c, c->nvec);
  if (st != DG_OK) return st;
  st = upload_elem_metrics(c);
  if (st != DG_OK) return st;
  if (c->cfg.fv) {
    const size_t nE = c->nElems, nS = c->nSides;
    if ((e = hipMalloc((void**)&c->d_fvV, nv * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&c->d_fvS, (size_t)9 * nE * c->N * c->n2 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&c->d_fvSb, 3 * nf * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&c->d_etype, nE * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void**)&c->d_etype_new, nE * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void**)&c->d_sidefv, nS * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void**)&c->d_efv, nE * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void**)&c->d_side_elem, 2 * nS * sizeof(int))) != hipSuccess) {
      free_device(c);
      return fail(c, e == hipErrorOutOfMemory ? DG_ERR_NOMEM : DG_ERR_HIP,
                  std::string("dg_upload_mesh: hipMalloc (FV): ") + hipGetErrorString(e));
    }
    std::vector<int> zeros(std::max(nE, nS), 0);
    HIPCHK(c, hipMemcpy(c->d_etype, zeros.data(), nE * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_etype_new, zeros.data(), nE * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_sidefv, zeros.data(), nS * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_efv, zeros.data(), nE * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_side_elem, c->side_elem.data(), 2 * nS * sizeof(int), hipMemcpyHostToDevice));
    st = build_fv(c);
    if (st != DG_OK) return st;
  }
  c->mesh_on_device = true;
  return DG_OK;
}

dg_status dg_upload_metrics(dg_ctx* c, const double* Ja, const double* sJ, const double* nvec) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_upload_metrics: null context");
  if (!c->mesh_on_device) return fail(c, DG_ERR_STATE, "dg_upload_metrics: no mesh on the device");
  if (!Ja || !sJ || !nvec) return fail(c, DG_ERR_ARG, "dg_upload_metrics: null pointer");
  const size_t nv = (size_t)c->nElems * c->n3, nf = (size_t)c->nSides * c->n2;
  for (size_t t = 0; t < nv; ++t)
    if (!(sJ[t] > 0.0) || !std::isfinite(sJ[t])) return fail(c, DG_ERR_MESH, "dg_upload_metrics: sJ must be positive");
  HIPCHK(c, hipMemcpy(c->d_Ja, Ja, 9 * nv * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_sJ, sJ, nv * sizeof(double), hipMemcpyHostToDevice));
  std::vector<double> nv3(nvec, nvec + 3 * nf);
  c->Ja.assign(Ja, Ja + 9 * nv);
  c->sJ.assign(sJ, sJ + nv);
  c->nvec = nv3;
  // |Omega| as dg_set_mesh sums it: per element, then in element order
  double vol = 0.0;
  const int n1 = c->n1, n3 = c->n3;
  for (int e = 0; e < c->nElems; ++e) {
    double ve = 0.0;
    for (int t = 0; t < n3; ++t) {
      int i = t % n1, j = (t / n1) % n1, k = t / (n1 * n1);
      size_t u = (size_t)e * n3 + t;
      c->wJ[u] = c->w[i] * c->w[j] * c->w[k] / sJ[u];
      ve += c->wJ[u];
    }
    vol += ve;
  }
  c->volume = vol;
  dg_status st = upload_face(c, nv3);
  if (st == DG_OK) st = upload_elem_metrics(c);
  if (st != DG_OK || !c->cfg.fv) return st;
  return build_fv(c);
}

dg_status dg_get_metrics(const dg_ctx* cc, double* xyz, double* Ja, double* sJ, double* nvec) {
  dg_ctx* c = const_cast<dg_ctx*>(cc);
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_get_metrics: null context");
  if (!c->mesh_set) return fail(c, DG_ERR_STATE, "dg_get_metrics: no mesh");
  if (xyz) std::memcpy(xyz, c->xyz.data(), c->xyz.size() * sizeof(double));
  if (Ja) std::memcpy(Ja, c->Ja.data(), c->Ja.size() * sizeof(double));
  if (sJ) std::memcpy(sJ, c->sJ.data(), c->sJ.size() * sizeof(double));
  if (nvec) std::memcpy(nvec, c->nvec.data(), c->nvec.size() * sizeof(double));
  return DG_OK;
}

dg_status dg_set_element_metrics(dg_ctx* c, int enable) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_set_element_metrics: null context");
  c->elem_metrics = enable != 0;
  return c->mesh_on_device ? upload_elem_metrics(c) : DG_OK;
}

dg_status dg_element_metric_count(const dg_ctx* c, int* count) {
  if (!c || !count) return fail(const_cast<dg_ctx*>(c), DG_ERR_ARG, "dg_element_metric_count: null pointer");
  if (!c->mesh_on_device) return fail(const_cast<dg_ctx*>(c), DG_ERR_STATE, "dg_element_metric_count: no mesh on the device");
  *count = c->n_const_metric;
  return DG_OK;
}

dg_status dg_node_coords(const dg_ctx* c, double* xyz_host) { return dg_get_metrics(c, xyz_host, nullptr, nullptr, nullptr); }

dg_status dg_sizes(const dg_ctx* cc, int* nElems, int* nSides, int* npe, size_t* state_len) {
  dg_ctx* c = const_cast<dg_ctx*>(cc);
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_sizes: null context");
  if (nElems) *nElems = c->nElems;
  if (nSides) *nSides = c->nSides;
  if (npe) *npe = c->n3;
  if (state_len) *state_len = (size_t)5 * c->nElems * c->n3;
  return DG_OK;
}

// ---------------------------------------------------------------------------
// Workspace
// ---------------------------------------------------------------------------
struct WsLayout {
  size_t utr[2], gtr, g, red, fvind, flag, total;
  // adjoint region: recomputed stage states Y_1..Y_{S-1}, forward RK
  // register, adjoint residual, face values of the gradient adjoint
  // (Navier-Stokes)
  size_t Y[DG_RK_MAX_STAGES - 1], dUf, aout, qbar, total_adjoint;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static int rk_stages(const dg_ctx* c) { return c->cfg.integrator == DG_RK_LSERK414 ? 14 : 5; }

// The context's scheme: coefficients into A, B (DG_RK_MAX_STAGES entries); returns S.
static int rk_scheme(const dg_ctx* c, double* A, double* B) {
  double C[DG_RK_MAX_STAGES];
  int ns = 0;
  dg_rk_coefficients(c->cfg.integrator, A, B, C, &ns);
  return ns;
}

static WsLayout ws_layout(const dg_ctx* c) {
  WsLayout L{};
  const size_t nf = (size_t)c->nSides * c->n2, nv = (size_t)c->nElems * c->n3;
  size_t off = 0;
  // U traces [2 slots][5][nf]; the split form on Gauss nodes appends the
  // traces' ln rho, ln beta [2 slots][2][nf]
  // (FV contexts: 10 values per face node, the DG trace or two primitive
  // sub-cell layers, then the logs of the split form on Gauss nodes)
  const bool es = c->cfg.volume_form == DG_FORM_SPLIT && c->cfg.nodes == DG_NODES_GAUSS;
  const int tv = (c->cfg.fv ? 10 : 5) + (es ? 2 : 0);
  for (int b = 0; b < 2; ++b) { L.utr[b] = off; off += align256(2 * (size_t)tv * nf * sizeof(double)); }
  const bool ns = c->cfg.physics == DG_PHYS_NAVIER_STOKES;
  // lifted face data [2 slots][12][nf]; FV contexts: the face-normal viscous
  // fluxes [2][4][nf], then the layer-0 sub-cell gradients [2][12][nf]
  L.gtr = off; off += ns ? align256(2 * (c->cfg.fv ? 16 : 12) * nf * sizeof(double)) : 0;
  L.g = off; off += ns ? align256(12 * nv * sizeof(double)) : 0;
  L.red = off; off += align256((size_t)(2 * reduction_blocks() + 8) * sizeof(double));
  L.fvind = off; off += c->cfg.fv ? align256((size_t)c->nElems * sizeof(double)) : 0;
  L.flag = off; off += 256;
  L.total = off;
  const size_t st = align256(5 * nv * sizeof(double));
  for (int k = 0; k + 1 < rk_stages(c); ++k) { L.Y[k] = off; off += st; }
  L.dUf = off; off += st;
  L.aout = off; off += st;
  L.qbar = off; off += ns ? align256(2 * 4 * nf * sizeof(double)) : 0;
  L.total_adjoint = off;
  return L;
}

size_t dg_workspace_bytes(const dg_ctx* c) {
  if (!c || !c->mesh_set) return 0;
  return ws_layout(c).total;
}

size_t dg_workspace_bytes_adjoint(const dg_ctx* c) {
  if (!c || !c->mesh_set) return 0;
  return ws_layout(c).total_adjoint;
}

dg_status dg_bind_workspace(dg_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_bind_workspace: null context");
  if (!c->mesh_set) return fail(c, DG_ERR_STATE, "dg_bind_workspace: no mesh");
  if (!dev_ptr) return fail(c, DG_ERR_ARG, "dg_bind_workspace: null pointer");
  if (((uintptr_t)dev_ptr & 255) != 0) return fail(c, DG_ERR_ARG, "dg_bind_workspace: pointer not 256-byte aligned");
  if (bytes < ws_layout(c).total) return fail(c, DG_ERR_ARG, "dg_bind_workspace: workspace too small");
  // a workspace of at least dg_workspace_bytes_adjoint also enables the adjoint calls
  c->ws = (char*)dev_ptr;
  c->ws_bytes = bytes;
  return DG_OK;
}

// ---------------------------------------------------------------------------
// Hot path
// ---------------------------------------------------------------------------
static dg_status ready(dg_ctx* c, const char* who) {
  if (!c) return fail(nullptr, DG_ERR_ARG, std::string(who) + ": null context");
  if (!c->mesh_on_device) return fail(c, DG_ERR_STATE, std::string(who) + ": no mesh uploaded");
  if (!c->ws) return fail(c, DG_ERR_STATE, std::string(who) + ": no workspace bound");
  return DG_OK;
}

static Cfg kcfg(const dg_ctx* c) {
  Cfg k;
  k.N = c->N; k.nodes = c->cfg.nodes; k.form = c->cfg.volume_form; k.physics = c->cfg.physics;
  k.precision = c->cfg.precision;
  k.roe = c->cfg.riemann == DG_RIEMANN_ROE ? 1 : 0;
  k.visc = c->cfg.viscosity == DG_VISC_SUTHERLAND ? 1 : 0;
  k.fv = c->cfg.fv;
  return k;
}

static Geo kgeo(const dg_ctx* c) {
  Geo g;
  g.nElems = c->nElems; g.nSides = c->nSides;
  g.Ja = c->d_Ja; g.sJ = c->d_sJ; g.em = c->d_em; g.face = c->d_face; g.efc = c->d_efc; g.basis = c->d_basis;
  g.etype = c->d_etype; g.sidefv = c->d_sidefv; g.efv = c->d_efv; g.fvV = c->d_fvV; g.fvS = c->d_fvS; g.fvSb = c->d_fvSb;
  return g;
}

static Work kwork(const dg_ctx* c) {
  WsLayout L = ws_layout(c);
  Work w;
  w.Utr[0] = (double*)(c->ws + L.utr[0]);
  w.Utr[1] = (double*)(c->ws + L.utr[1]);
  const bool ns = c->cfg.physics == DG_PHYS_NAVIER_STOKES;
  w.gtr = ns ? (double*)(c->ws + L.gtr) : nullptr;
  w.g = ns ? (double*)(c->ws + L.g) : nullptr;
  w.red = (double*)(c->ws + L.red);
  w.flag = (int*)(c->ws + L.flag);
  return w;
}

#define LAUNCHCHK(ctx, call)                                                                          \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) return fail(ctx, DG_ERR_HIP, std::string("launch ") + #call + ": " + hipGetErrorString(e_)); \
  } while (0)

// One residual evaluation whose traces of U already sit in Utr[cur].
static dg_status stage(dg_ctx* c, int mode, const double* U, double* Ut, double* Uio, double* dU, int cur, double A,
                       double B, double dt, hipStream_t s) {
  Cfg k = kcfg(c);
  Geo g = kgeo(c);
  Work w = kwork(c);
  if (c->cfg.physics == DG_PHYS_NAVIER_STOKES) {
    ProfScope ps(c, FAM_LIFT, s);
    LAUNCHCHK(c, launch_lift(k, 1, g, c->phys, U, w.Utr[cur], w.g, w.gtr, s));
  }
  {
    ProfScope ps(c, FAM_VOLUME, s);
    LAUNCHCHK(c, launch_volume(k, g, c->phys, mode, U, w.Utr[cur], w.g, w.gtr, Ut, Uio, dU, w.Utr[cur ^ 1], A, B, dt, s));
  }
  if (c->cfg.fv) {
    // FV elements (the volume kernel above leaves them untouched)
    ProfScope ps(c, FAM_FV, s);
    LAUNCHCHK(c, launch_fv(k, g, c->phys, mode, U, w.Utr[cur], w.g, w.gtr, Ut, Uio, dU, w.Utr[cur ^ 1], A, B, dt, s));
  }
  return DG_OK;
}

// Face traces of U into Utr (the FV context's two-layer traces on FV faces).
static dg_status traces(dg_ctx* c, const double* U, double* Utr, hipStream_t s) {
  ProfScope ps(c, FAM_TRACE, s);
  if (c->cfg.fv) LAUNCHCHK(c, launch_trace_fv(kcfg(c), kgeo(c), c->phys, U, Utr, s));
  else LAUNCHCHK(c, launch_trace(kcfg(c), kgeo(c), c->phys, U, Utr, s));
  return DG_OK;
}

dg_status dg_rhs(dg_ctx* c, const double* U, double* Ut, double t, void* stream) {
  dg_status st = ready(c, "dg_rhs");
  if (st != DG_OK) return st;
  if (!U || !Ut) return fail(c, DG_ERR_ARG, "dg_rhs: null pointer");
  if (U == Ut) return fail(c, DG_ERR_ARG, "dg_rhs: U and Ut alias");
  (void)t;
  hipStream_t s = (hipStream_t)stream;
  Work w = kwork(c);
  st = traces(c, U, w.Utr[0], s);
  if (st != DG_OK) return st;
  return stage(c, 0, U, Ut, nullptr, nullptr, 0, 0.0, 0.0, 0.0, s);
}

dg_status dg_lift(dg_ctx* c, const double* U, double* gout, void* stream) {
  dg_status st = ready(c, "dg_lift");
  if (st != DG_OK) return st;
  if (!U || !gout) return fail(c, DG_ERR_ARG, "dg_lift: null pointer");
  if (c->cfg.physics != DG_PHYS_NAVIER_STOKES) return fail(c, DG_ERR_ARG, "dg_lift: Navier-Stokes contexts only");
  if (c->cfg.fv) return fail(c, DG_ERR_UNSUPPORTED, "dg_lift: contexts with FV sub-cells are not covered");
  hipStream_t s = (hipStream_t)stream;
  Work w = kwork(c);
  LAUNCHCHK(c, launch_trace(kcfg(c), kgeo(c), c->phys, U, w.Utr[0], s));
  LAUNCHCHK(c, launch_lift(kcfg(c), 0, kgeo(c), c->phys, U, w.Utr[0], gout, w.gtr, s));
  return DG_OK;
}

dg_status dg_rk_step(dg_ctx* c, double* U, double* dU, double t, double dt, int nsteps, void* stream) {
  dg_status st = ready(c, "dg_rk_step");
  if (st != DG_OK) return st;
  if (!U || !dU) return fail(c, DG_ERR_ARG, "dg_rk_step: null pointer");
  if (U == dU) return fail(c, DG_ERR_ARG, "dg_rk_step: U and dU alias");
  if (nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return fail(c, DG_ERR_ARG, "dg_rk_step: nsteps/dt");
  (void)t;
  if (nsteps == 0) return DG_OK;
  hipStream_t s = (hipStream_t)stream;
  double A[DG_RK_MAX_STAGES], B[DG_RK_MAX_STAGES];
  const int ns = rk_scheme(c, A, B);
  Work w = kwork(c);
  const size_t n = (size_t)5 * c->nElems * c->n3;
  {
    ProfScope ps(c, FAM_OTHER, s);
    LAUNCHCHK(c, launch_fill(dU, n, 0.0, s));
  }
  st = traces(c, U, w.Utr[0], s);
  if (st != DG_OK) return st;
  int cur = 0;
  for (int step = 0; step < nsteps; ++step)
    for (int k = 0; k < ns; ++k) {
      st = stage(c, 1, U, nullptr, U, dU, cur, A[k], B[k], dt, s);
      if (st != DG_OK) return st;
      cur ^= 1;
    }
  return DG_OK;
}

dg_status dg_rk_step_stages(dg_ctx* c, double* U, double* dU, double t, double dt, double* Y, void* stream) {
  dg_status st = ready(c, "dg_rk_step_stages");
  if (st != DG_OK) return st;
  if (!U || !dU || !Y) return fail(c, DG_ERR_ARG, "dg_rk_step_stages: null pointer");
  if (U == dU || Y == U || Y == dU) return fail(c, DG_ERR_ARG, "dg_rk_step_stages: aliasing arrays");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, DG_ERR_ARG, "dg_rk_step_stages: dt");
  if (c->cfg.fv) return fail(c, DG_ERR_UNSUPPORTED, "dg_rk_step_stages: contexts with FV sub-cells are not covered");
  (void)t;
  hipStream_t s = (hipStream_t)stream;
  double A[DG_RK_MAX_STAGES], B[DG_RK_MAX_STAGES];
  const int ns = rk_scheme(c, A, B);
  Work w = kwork(c);
  const size_t n = (size_t)5 * c->nElems * c->n3;
  {
    ProfScope ps(c, FAM_OTHER, s);
    LAUNCHCHK(c, launch_fill(dU, n, 0.0, s));
  }
  st = traces(c, U, w.Utr[0], s);
  if (st != DG_OK) return st;
  // stage k reads its input (U, then Y_k) and writes the next stage's input
  // (Y_{k+1}, the last one U): the same arithmetic as in place
  int cur = 0;
  for (int k = 0; k < ns; ++k) {
    const double* in = k == 0 ? U : Y + (size_t)(k - 1) * n;
    double* outp = k == ns - 1 ? U : Y + (size_t)k * n;
    st = stage(c, 1, in, nullptr, outp, dU, cur, A[k], B[k], dt, s);
    if (st != DG_OK) return st;
    cur ^= 1;
  }
  return DG_OK;
}

dg_status dg_rk_step_noalloc(dg_ctx* c, double* U, double* dU, double t, double dt, int nsteps, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_rk_step_noalloc: null context");
  if (!c->mesh_on_device) return fail(c, DG_ERR_STATE, "dg_rk_step_noalloc: no mesh uploaded");
  const size_t need = ws_layout(c).total;
  if (need > kStaticScratchBytes) {
    char buf[192];
    std::snprintf(buf, sizeof buf, "dg_rk_step_noalloc: the mesh needs %zu bytes of scratch, above the static %zu",
                  need, kStaticScratchBytes);
    return fail(c, DG_ERR_ARG, buf);
  }
  void* scr = nullptr;
  HIPCHK(c, static_scratch(&scr));
  // Run dg_rk_step on the static scratch in place of the bound workspace, with
  // event profiling off (no event creation), and restore both afterwards.
  struct Swap {
    dg_ctx* c; char* ws; size_t bytes; bool prof;
    ~Swap() { c->ws = ws; c->ws_bytes = bytes; c->prof = prof; }
  } keep{c, c->ws, c->ws_bytes, c->prof};
  c->ws = (char*)scr;
  c->ws_bytes = kStaticScratchBytes;
  c->prof = false;
  dg_status st = dg_rk_step(c, U, dU, t, dt, nsteps, stream);
  if (st != DG_OK) {
    std::string m = c->err;
    c->err = "dg_rk_step_noalloc: " + m;
  }
  return st;
}

static dg_status ready_adjoint(dg_ctx* c, const char* who) {
  dg_status st = ready(c, who);
  if (st != DG_OK) return st;
  if (c->cfg.precision != DG_PREC_FP64) return fail(c, DG_ERR_UNSUPPORTED, std::string(who) + ": FP64 contexts only");
  if (c->cfg.fv) return fail(c, DG_ERR_UNSUPPORTED, std::string(who) + ": the adjoint does not cover FV sub-cells");
  if (c->ws_bytes < ws_layout(c).total_adjoint)
    return fail(c, DG_ERR_STATE, std::string(who) + ": bound workspace is smaller than dg_workspace_bytes_adjoint");
  return DG_OK;
}

// out = (dR/dU(U))^T lam, with the forward traces (and gradients) of U recomputed.
static dg_status adjoint_residual(dg_ctx* c, const double* U, const double* lam, double* out, hipStream_t s,
                                  const AdjUpd& up = AdjUpd{nullptr, nullptr, 0.0, 0.0, 0.0}) {
  Cfg k = kcfg(c);
  Geo g = kgeo(c);
  Work w = kwork(c);
  WsLayout L = ws_layout(c);
  double* qbar = k.physics == DG_PHYS_NAVIER_STOKES ? (double*)(c->ws + L.qbar) : nullptr;
  {
    ProfScope ps(c, FAM_TRACE, s);
    LAUNCHCHK(c, launch_trace(k, g, c->phys, U, w.Utr[0], s));
  }
  if (k.physics == DG_PHYS_NAVIER_STOKES) {
    ProfScope ps(c, FAM_LIFT, s);
    LAUNCHCHK(c, launch_lift(k, 0, g, c->phys, U, w.Utr[0], w.g, w.gtr, s));
  }
  ProfScope ps(c, FAM_ADJOINT, s);
  LAUNCHCHK(c, launch_adjoint(k, g, c->phys, U, lam, w.Utr[0], w.Utr[1], w.g, w.gtr, out, qbar, up, s));
  return DG_OK;
}

dg_status dg_adjoint_rhs(dg_ctx* c, const double* U, const double* lam, double* out, void* stream) {
  dg_status st = ready_adjoint(c, "dg_adjoint_rhs");
  if (st != DG_OK) return st;
  if (!U || !lam || !out) return fail(c, DG_ERR_ARG, "dg_adjoint_rhs: null pointer");
  if (out == U || out == lam) return fail(c, DG_ERR_ARG, "dg_adjoint_rhs: out aliases an input");
  return adjoint_residual(c, U, lam, out, (hipStream_t)stream);
}

// Reverse sweep of one RK step over the stage inputs Y[0..S-1]:
// lamdU = B_{S-1} lamU; per stage s: lamU += dt J(Y_s)^T lamdU; lamdU = A_s lamdU + B_{s-1} lamU.
static dg_status reverse_sweep(dg_ctx* c, const double* const* Y, double* lamU, double* lamdU, double dt,
                               hipStream_t s) {
  double A[DG_RK_MAX_STAGES], B[DG_RK_MAX_STAGES];
  const int ns = rk_scheme(c, A, B);
  const size_t n = (size_t)5 * c->nElems * c->n3;
  double* aout = (double*)(c->ws + ws_layout(c).aout);
  {
    ProfScope ps(c, FAM_OTHER, s);
    LAUNCHCHK(c, launch_scale_copy(n, lamU, lamdU, B[ns - 1], s));
  }
  // (the update is fused into the stage's last adjoint kernel, which for
  // Navier-Stokes also writes the next stage's surface adjoint into Lbar:
  // nothing else touches that buffer before the next stage reads it)
  const bool visc = c->cfg.physics == DG_PHYS_NAVIER_STOKES;
  double* Lbar = kwork(c).Utr[1];
  for (int k = ns - 1; k >= 0; --k) {
    AdjUpd up{lamU, lamdU, dt, A[k], k > 0 ? B[k - 1] : 0.0};
    up.Lnext = visc && k > 0 ? Lbar : nullptr;
    up.lbar_ready = visc && k < ns - 1 ? 1 : 0;
    dg_status st = adjoint_residual(c, Y[k], lamdU, aout, s, up);
    if (st != DG_OK) return st;
  }
  return DG_OK;
}

static dg_status adjoint_step_checks(dg_ctx* c, const char* who, const double* Un, double* lamU, double* lamdU,
                                     double dt) {
  dg_status st = ready_adjoint(c, who);
  if (st != DG_OK) return st;
  if (!Un || !lamU || !lamdU) return fail(c, DG_ERR_ARG, std::string(who) + ": null pointer");
  if (lamU == lamdU || Un == lamU || Un == lamdU) return fail(c, DG_ERR_ARG, std::string(who) + ": aliasing arrays");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, DG_ERR_ARG, std::string(who) + ": dt");
  return DG_OK;
}

dg_status dg_adjoint_rk_step(dg_ctx* c, const double* Un, double* lamU, double* lamdU, double t, double dt,
                             void* stream) {
  dg_status st = adjoint_step_checks(c, "dg_adjoint_rk_step", Un, lamU, lamdU, dt);
  if (st != DG_OK) return st;
  (void)t;
  hipStream_t s = (hipStream_t)stream;
  double A[DG_RK_MAX_STAGES], B[DG_RK_MAX_STAGES];
  const int ns = rk_scheme(c, A, B);
  WsLayout L = ws_layout(c);
  Work w = kwork(c);
  const size_t n = (size_t)5 * c->nElems * c->n3;
  const double* Y[DG_RK_MAX_STAGES];
  Y[0] = Un;
  for (int k = 0; k + 1 < ns; ++k) Y[k + 1] = (const double*)(c->ws + L.Y[k]);
  double* dUf = (double*)(c->ws + L.dUf);
  // recompute the stage inputs Y_1..Y_{S-1} of this step
  {
    ProfScope ps(c, FAM_OTHER, s);
    LAUNCHCHK(c, launch_fill(dUf, n, 0.0, s));
  }
  {
    ProfScope ps(c, FAM_TRACE, s);
    LAUNCHCHK(c, launch_trace(kcfg(c), kgeo(c), c->phys, Un, w.Utr[0], s));
  }
  int cur = 0;
  for (int k = 0; k + 1 < ns; ++k) {
    st = stage(c, 1, Y[k], nullptr, const_cast<double*>(Y[k + 1]), dUf, cur, A[k], B[k], dt, s);
    if (st != DG_OK) return st;
    cur ^= 1;
  }
  return reverse_sweep(c, Y, lamU, lamdU, dt, s);
}

dg_status dg_adjoint_rk_step_stages(dg_ctx* c, const double* Un, const double* Ystages, double* lamU, double* lamdU,
                                    double t, double dt, void* stream) {
  dg_status st = adjoint_step_checks(c, "dg_adjoint_rk_step_stages", Un, lamU, lamdU, dt);
  if (st != DG_OK) return st;
  if (!Ystages) return fail(c, DG_ERR_ARG, "dg_adjoint_rk_step_stages: null pointer");
  if (Ystages == lamU || Ystages == lamdU) return fail(c, DG_ERR_ARG, "dg_adjoint_rk_step_stages: aliasing arrays");
  (void)t;
  double A[DG_RK_MAX_STAGES], B[DG_RK_MAX_STAGES];
  const int ns = rk_scheme(c, A, B);
  const size_t n = (size_t)5 * c->nElems * c->n3;
  const double* Y[DG_RK_MAX_STAGES];
  Y[0] = Un;
  for (int k = 0; k + 1 < ns; ++k) Y[k + 1] = Ystages + (size_t)k * n;
  return reverse_sweep(c, Y, lamU, lamdU, dt, (hipStream_t)stream);
}

dg_status dg_kinetic_energy(dg_ctx* c, const double* U, double rho0U0sq, double* out_dev, void* stream) {
  dg_status st = ready(c, "dg_kinetic_energy");
  if (st != DG_OK) return st;
  if (!U || !out_dev) return fail(c, DG_ERR_ARG, "dg_kinetic_energy: null pointer");
  if (!(rho0U0sq > 0.0)) return fail(c, DG_ERR_ARG, "dg_kinetic_energy: rho0U0sq must be positive");
  Work w = kwork(c);
  LAUNCHCHK(c, launch_kinetic_energy(kcfg(c), kgeo(c), U, w.red, out_dev, 1.0 / (2.0 * rho0U0sq * c->volume),
                                     (hipStream_t)stream));
  return DG_OK;
}

dg_status dg_kinetic_energy_grad(dg_ctx* c, const double* U, double rho0U0sq, double scale, double* grad,
                                 void* stream) {
  dg_status st = ready(c, "dg_kinetic_energy_grad");
  if (st != DG_OK) return st;
  if (!U || !grad) return fail(c, DG_ERR_ARG, "dg_kinetic_energy_grad: null pointer");
  if (!(rho0U0sq > 0.0)) return fail(c, DG_ERR_ARG, "dg_kinetic_energy_grad: rho0U0sq must be positive");
  LAUNCHCHK(c, launch_kinetic_energy_grad(kcfg(c), kgeo(c), U, grad, scale / (2.0 * rho0U0sq * c->volume),
                                          (hipStream_t)stream));
  return DG_OK;
}

dg_status dg_timestep(dg_ctx* c, const double* U, double cfl, double* dt_out, void* stream) {
  dg_status st = ready(c, "dg_timestep");
  if (st != DG_OK) return st;
  if (!U || !dt_out) return fail(c, DG_ERR_ARG, "dg_timestep: null pointer");
  if (!(cfl > 0.0)) return fail(c, DG_ERR_ARG, "dg_timestep: cfl must be positive");
  hipStream_t s = (hipStream_t)stream;
  Work w = kwork(c);
  double* out2 = w.red + 2 * reduction_blocks();
  LAUNCHCHK(c, launch_timestep(kcfg(c), kgeo(c), c->phys, U, w.red, out2, s));
  double h[2];
  HIPCHK(c, hipMemcpyAsync(h, out2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (!(h[0] > 0.0) || !std::isfinite(h[0])) return fail(c, DG_ERR_NONPHYSICAL, "dg_timestep: no finite wave speed");
  // advective limit ~ 1/(N+1)^2 above N = 3, viscous limit ~ 1/(N+1)^4: the
  // growth of the DG operator's spectral radius; the constants keep LSERK4(5)
  // linearly stable for N = 1..7 at cfl = 0.9.  LSERK4-14's stability limit
  // on the same spectra is 3.98 times larger; it takes 3.75 times the step.
  const double n1 = c->N + 1.0;
  const double sc = cfl * (c->cfg.integrator == DG_RK_LSERK414 ? 3.75 : 1.0);
  double dt = sc * std::min(2.0 / n1, 8.0 / (n1 * n1)) / h[0];
  if (c->cfg.physics == DG_PHYS_NAVIER_STOKES && h[1] > 0.0) dt = std::min(dt, sc * 32.0 / (n1 * n1 * n1 * n1 * h[1]));
  *dt_out = dt;
  return DG_OK;
}

dg_status dg_init_state(dg_ctx* c, const double* U_src, int src_is_device, double* U, void* stream) {
  dg_status st = ready(c, "dg_init_state");
  if (st != DG_OK) return st;
  if (!U_src || !U) return fail(c, DG_ERR_ARG, "dg_init_state: null pointer");
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = sizeof(double) * 5 * (size_t)c->nElems * c->n3;
  if (U_src != U) {
    HIPCHK(c, hipMemcpyAsync(U, U_src, bytes, src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  }
  return dg_check_state(c, U, stream);
}

dg_status dg_check_state(dg_ctx* c, const double* U, void* stream) {
  dg_status st = ready(c, "dg_check_state");
  if (st != DG_OK) return st;
  if (!U) return fail(c, DG_ERR_ARG, "dg_check_state: null pointer");
  hipStream_t s = (hipStream_t)stream;
  Work w = kwork(c);
  LAUNCHCHK(c, launch_fill_int(w.flag, 1, 0, s));
  LAUNCHCHK(c, launch_check_state(kcfg(c), kgeo(c), c->phys, U, w.flag, s));
  int h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (h) return fail(c, DG_ERR_NONPHYSICAL, "dg_check_state: rho <= 0, p <= 0 or non-finite value found");
  return DG_OK;
}

// ---------------------------------------------------------------------------
// FV sub-cells: switching and indicator
// ---------------------------------------------------------------------------
static dg_status ready_fv(dg_ctx* c, const char* who) {
  dg_status st = ready(c, who);
  if (st != DG_OK) return st;
  if (!c->cfg.fv) return fail(c, DG_ERR_STATE, std::string(who) + ": the context was created without fv");
  return DG_OK;
}

// Converts U/dU to the types in d_etype_new, sets d_etype, then the side flags.
static dg_status fv_apply(dg_ctx* c, double* U, double* dU, hipStream_t s) {
  ProfScope ps(c, FAM_OTHER, s);
  LAUNCHCHK(c, launch_fv_switch(kcfg(c), kgeo(c), U, dU, c->d_etype_new, c->d_etype, s));
  LAUNCHCHK(c, launch_fv_side_flags(c->nSides, c->d_side_elem, c->d_etype, c->d_sidefv, s));
  LAUNCHCHK(c, launch_fv_elem_flags(c->nElems, c->d_efc, c->d_sidefv, c->d_etype, c->d_efv, s));
  return DG_OK;
}

dg_status dg_fv_switch(dg_ctx* c, double* U, double* dU, const int* mask_host, void* stream) {
  dg_status st = ready_fv(c, "dg_fv_switch");
  if (st != DG_OK) return st;
  if (!U || !mask_host) return fail(c, DG_ERR_ARG, "dg_fv_switch: null pointer");
  if (U == dU) return fail(c, DG_ERR_ARG, "dg_fv_switch: U and dU alias");
  std::vector<int> m(mask_host, mask_host + c->nElems);
  for (int& v : m) {
    if (v != 0 && v != 1) return fail(c, DG_ERR_ARG, "dg_fv_switch: mask entries must be 0 or 1");
  }
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(c, hipMemcpyAsync(c->d_etype_new, m.data(), m.size() * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return fv_apply(c, U, dU, s);
}

dg_status dg_fv_indicator(dg_ctx* c, const double* U, double* ind_dev, void* stream) {
  dg_status st = ready_fv(c, "dg_fv_indicator");
  if (st != DG_OK) return st;
  if (!U || !ind_dev) return fail(c, DG_ERR_ARG, "dg_fv_indicator: null pointer");
  hipStream_t s = (hipStream_t)stream;
  ProfScope ps(c, FAM_OTHER, s);
  LAUNCHCHK(c, launch_fv_indicator(kcfg(c), kgeo(c), U, ind_dev, s));
  return DG_OK;
}

dg_status dg_fv_switch_by_indicator(dg_ctx* c, double* U, double* dU, double lo, double hi, void* stream) {
  dg_status st = ready_fv(c, "dg_fv_switch_by_indicator");
  if (st != DG_OK) return st;
  if (!U) return fail(c, DG_ERR_ARG, "dg_fv_switch_by_indicator: null pointer");
  if (U == dU) return fail(c, DG_ERR_ARG, "dg_fv_switch_by_indicator: U and dU alias");
  if (!(lo <= hi)) return fail(c, DG_ERR_ARG, "dg_fv_switch_by_indicator: need ind_lo <= ind_hi");
  hipStream_t s = (hipStream_t)stream;
  double* ind = (double*)(c->ws + ws_layout(c).fvind);
  {
    ProfScope ps(c, FAM_OTHER, s);
    LAUNCHCHK(c, launch_fv_indicator(kcfg(c), kgeo(c), U, ind, s));
    LAUNCHCHK(c, launch_fv_decide(c->nElems, ind, lo, hi, c->d_etype, c->d_etype_new, s));
  }
  return fv_apply(c, U, dU, s);
}

dg_status dg_fv_mask(dg_ctx* c, int* mask_host, void* stream) {
  dg_status st = ready_fv(c, "dg_fv_mask");
  if (st != DG_OK) return st;
  if (!mask_host) return fail(c, DG_ERR_ARG, "dg_fv_mask: null pointer");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(c, hipMemcpyAsync(mask_host, c->d_etype, (size_t)c->nElems * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return DG_OK;
}

dg_status dg_profile(dg_ctx* c, int enable) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_profile: null context");
  prof_collect(c);
  for (int f = 0; f < 6; ++f) { c->prof_ms[f] = 0.0; c->prof_n[f] = 0; }
  c->prof = enable != 0;
  c->prof_mask = 0x3f;
  return DG_OK;
}

dg_status dg_profile_families(dg_ctx* c, int mask) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_profile_families: null context");
  if (mask < 0 || mask > 0x3f) return fail(c, DG_ERR_ARG, "dg_profile_families: mask outside 0..63");
  prof_collect(c);
  for (int f = 0; f < 6; ++f) { c->prof_ms[f] = 0.0; c->prof_n[f] = 0; }
  c->prof = mask != 0;
  c->prof_mask = mask;
  return DG_OK;
}

dg_status dg_profile_query(dg_ctx* c, const char* kernel, double* total_ms, long* count) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "dg_profile_query: null context");
  if (!kernel || !total_ms || !count) return fail(c, DG_ERR_ARG, "dg_profile_query: null pointer");
  int fam = -1;
  for (int f = 0; f < 6; ++f)
    if (std::strcmp(kernel, kFamNames[f]) == 0) fam = f;
  if (fam < 0) return fail(c, DG_ERR_ARG, std::string("dg_profile_query: unknown kernel family ") + kernel);
  prof_collect(c);
  *total_ms = c->prof_ms[fam];
  *count = c->prof_n[fam];
  return DG_OK;
}

}  // extern "C"

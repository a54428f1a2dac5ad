// Drives every exported oracle routine on small periodic meshes, for the
// AddressSanitizer / UndefinedBehaviorSanitizer build of the oracle (CPU).
// Exits non-zero if a result is not finite; the sanitizers abort on a
// memory or undefined-behaviour error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
const char* orc_last_error();
int orc_basis(int, int, double*, double*, double*, double*, double*, double*);
void* orc_create(const int*, const double*, int, int, const double*, int, const int*, const int*, const int*);
int orc_check_jacobians(void*);
void orc_destroy(void*);
int orc_rk_coeffs(int, double*, double*, double*);
void orc_geometry(void*, double*, double*, double*);
int orc_geometry_sample(void*, int, const int*, double*, double*, double*);
void orc_face_normals(void*, double*);
int orc_rhs(void*, const double*, double*, double);
int orc_rhs_elems(void*, const double*, double*, double, int, const int*);
int orc_rhs_sample(void*, const double*, double*, double, int, const int*);
int orc_lift(void*, const double*, double*);
int orc_rhs_jvp(void*, const double*, const double*, double*, double*, double);
int orc_lserk(void*, double*, int, double, double);
int orc_lserk_jvp(void*, double*, double*, int, double, double);
double orc_kinetic_energy(void*, const double*, double);
double orc_kinetic_energy_jvp(void*, const double*, const double*, double);
double orc_timestep(void*, const double*, double);
int orc_rhs_vjp(void*, const double*, const double*, double*, double);
int orc_kinetic_energy_grad(void*, const double*, double, double*);
int orc_lserk_adjoint(void*, const double*, double*, int, double, double);
int orc_rhs_opcount(void*, const double*, uint64_t*);
int orc_fv_set_mask(void*, const int*);
int orc_fv_switch(void*, double*, double*, const int*);
void orc_fv_get_mask(void*, int*);
int orc_fv_indicator(void*, const double*, double*);
int orc_fv_geometry(void*, double*, double*, double*);
int orc_fv_operators(void*, double*, double*, double*);
int orc_fv_convert(void*, int, int, const double*, double*);
int orc_opcount_point(int, const double*, const double*, const double*, const double*, uint64_t*);
double orc_logmean(double, double);
}

static int g_bad = 0;
static void finite(const std::vector<double>& v, const char* what) {
  for (double x : v)
    if (!std::isfinite(x)) { std::fprintf(stderr, "non-finite result in %s\n", what); g_bad = 1; return; }
}

struct Mesh {
  int nE, Ng, nS;
  std::vector<double> X;
  std::vector<int> se, sl, so;
};

// Periodic Kx x Ky x Kz box on [-pi, pi]^3, equispaced geometry nodes, optional curved displacement.
static Mesh box(int Kx, int Ky, int Kz, int Ng, double amp) {
  Mesh m;
  m.nE = Kx * Ky * Kz; m.Ng = Ng; m.nS = 3 * m.nE;
  const int g1 = Ng + 1;
  m.X.assign((size_t)3 * m.nE * g1 * g1 * g1, 0.0);
  const double pi = std::acos(-1.0), h[3] = {2 * pi / Kx, 2 * pi / Ky, 2 * pi / Kz};
  for (int kz = 0; kz < Kz; ++kz)
    for (int ky = 0; ky < Ky; ++ky)
      for (int kx = 0; kx < Kx; ++kx) {
        const int e = (kz * Ky + ky) * Kx + kx;
        for (int c = 0; c < g1; ++c)
          for (int b = 0; b < g1; ++b)
            for (int a = 0; a < g1; ++a) {
              const double x = -pi + (kx + (double)a / Ng) * h[0], y = -pi + (ky + (double)b / Ng) * h[1],
                           z = -pi + (kz + (double)c / Ng) * h[2];
              const double bump = amp * std::sin(x) * std::sin(y) * std::sin(z);
              const size_t o = (size_t)e * g1 * g1 * g1 + (c * g1 + b) * g1 + a;
              m.X[o] = x + bump;
              m.X[(size_t)m.nE * g1 * g1 * g1 + o] = y + bump;
              m.X[(size_t)2 * m.nE * g1 * g1 * g1 + o] = z + bump;
            }
        const int nb[3] = {(kz * Ky + ky) * Kx + (kx + 1) % Kx, (kz * Ky + (ky + 1) % Ky) * Kx + kx,
                           (((kz + 1) % Kz) * Ky + ky) * Kx + kx};
        for (int d = 0; d < 3; ++d) {
          m.se.push_back(e); m.se.push_back(nb[d]);
          m.sl.push_back(2 * d + 1); m.sl.push_back(2 * d);
          m.so.push_back(0);
        }
      }
  return m;
}

static void exercise(const int* icfg, const double* dcfg, const Mesh& m) {
  void* h = orc_create(icfg, dcfg, m.nE, m.Ng, m.X.data(), m.nS, m.se.data(), m.sl.data(), m.so.data());
  if (!h) { std::fprintf(stderr, "orc_create: %s\n", orc_last_error()); g_bad = 1; return; }
  const int N = icfg[0], n1 = N + 1, n3 = n1 * n1 * n1, n2 = n1 * n1;
  const size_t n = (size_t)5 * m.nE * n3;
  if (orc_check_jacobians(h)) g_bad = 1;
  std::vector<double> xyz((size_t)3 * m.nE * n3), J((size_t)m.nE * n3), Ja((size_t)9 * m.nE * n3), nv((size_t)3 * m.nS * n2);
  orc_geometry(h, xyz.data(), J.data(), Ja.data());
  orc_face_normals(h, nv.data());
  finite(Ja, "geometry");
  std::vector<double> U(n), R(n), dU(n), dR(n), lam(n), out(n), g((size_t)12 * m.nE * n3);
  for (size_t i = 0; i < n; ++i) {
    const size_t v = i / ((size_t)m.nE * n3), p = i % ((size_t)m.nE * n3);
    const double s = std::sin(0.37 * p + 0.11 * v);
    U[i] = v == 0 ? 1.0 + 0.1 * s : (v == 4 ? 2.6 + 0.1 * s : 0.1 * s);
    dU[i] = std::cos(0.23 * i);
    lam[i] = std::sin(0.19 * i);
  }
  if (icfg[10]) {
    std::vector<int> mask(m.nE);
    for (int e = 0; e < m.nE; ++e) mask[e] = e % 2;
    orc_fv_switch(h, U.data(), nullptr, mask.data());
    std::vector<int> got(m.nE);
    orc_fv_get_mask(h, got.data());
    std::vector<double> V((size_t)m.nE * n3), Si((size_t)m.nE * 9 * N * n2), Sb((size_t)m.nS * 3 * n2);
    orc_fv_geometry(h, V.data(), Si.data(), Sb.data());
    std::vector<double> B(n2), Bi(n2), Vi(n2), blk((size_t)5 * n3), blk2((size_t)5 * n3);
    orc_fv_operators(h, B.data(), Bi.data(), Vi.data());
    for (int x = 0; x < 5 * n3; ++x) blk[x] = U[(size_t)(x / n3) * m.nE * n3 + x % n3];
    orc_fv_convert(h, 0, 0, blk.data(), blk2.data());
    orc_fv_convert(h, 0, 1, blk2.data(), blk.data());
    std::vector<double> ind(m.nE);
    orc_fv_indicator(h, U.data(), ind.data());
    finite(V, "fv geometry");
  }
  orc_rhs(h, U.data(), R.data(), 0.0);
  finite(R, "rhs");
  const int list[2] = {m.nE - 1, 0};
  std::vector<double> smp((size_t)5 * 2 * n3);
  if (orc_rhs_sample(h, U.data(), smp.data(), 0.0, 2, list)) g_bad = 1;
  orc_rhs_elems(h, U.data(), R.data(), 0.0, 2, list);
  std::vector<double> gx((size_t)3 * 2 * n3), gj((size_t)2 * n3), gja((size_t)9 * 2 * n3);
  orc_geometry_sample(h, 2, list, gx.data(), gj.data(), gja.data());
  if (icfg[3] == 1) { orc_lift(h, U.data(), g.data()); finite(g, "lift"); }
  orc_rhs_jvp(h, U.data(), dU.data(), R.data(), dR.data(), 0.0);
  finite(dR, "jvp");
  orc_rhs_vjp(h, U.data(), lam.data(), out.data(), 0.0);
  finite(out, "vjp");
  uint64_t cnt[5];
  orc_rhs_opcount(h, U.data(), cnt);
  const double dt = orc_timestep(h, U.data(), 0.9);
  std::vector<double> U1 = U, D1 = dU;
  orc_lserk(h, U1.data(), 2, dt, 0.0);
  orc_lserk_jvp(h, U1.data(), D1.data(), 1, dt, 0.0);
  finite(U1, "lserk");
  if (!icfg[10]) {
    std::vector<double> lamU = lam;
    orc_lserk_adjoint(h, U.data(), lamU.data(), 2, dt, 0.0);
    finite(lamU, "lserk adjoint");
  }
  std::vector<double> ge(n);
  orc_kinetic_energy(h, U.data(), 1.0);
  orc_kinetic_energy_jvp(h, U.data(), dU.data(), 1.0);
  orc_kinetic_energy_grad(h, U.data(), 1.0, ge.data());
  orc_destroy(h);
}

int main() {
  const Mesh affine = box(2, 2, 1, 1, 0.0), curved = box(2, 1, 2, 3, 0.1);
  // icfg = {N, nodes, form, physics, twopoint, dissipation, mms, integrator, viscosity, hybrid, fv}
  const int cfgs[][11] = {
      {3, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0}, {3, 1, 1, 1, 0, 1, 0, 1, 0, 0, 0}, {2, 0, 1, 1, 0, 1, 0, 0, 0, 0, 0},
      {3, 1, 1, 1, 0, 2, 0, 0, 1, 0, 0}, {2, 1, 0, 1, 1, 0, 1, 0, 0, 0, 0}, {3, 1, 1, 0, 0, 1, 0, 0, 0, 1, 0},
      {2, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1}, {3, 1, 1, 0, 0, 1, 0, 0, 0, 0, 1}};
  const double dcfg[8] = {1.4, 0.05, 0.72, 1.0, 0.1, 1.0, 1.0, 0.4};
  for (const auto& c : cfgs) {
    exercise(c, dcfg, affine);
    exercise(c, dcfg, curved);
  }
  // point routines and bad input
  double x[8], w[8], D[64], Lm[8], Lp[8], DS[64], A[14], B[14], C[14];
  orc_basis(7, 1, x, w, D, Lm, Lp, DS);
  orc_rk_coeffs(1, A, B, C);
  const double Ua[5] = {1.0, 0.1, 0.2, 0.3, 3.0}, Ub[5] = {1.5, 0.1, 0.2, 0.3, 4.0}, nn[3] = {0.3, 0.4, 0.5};
  uint64_t cnt[5];
  for (int k = 0; k < 3; ++k) orc_opcount_point(k, dcfg, Ua, Ub, nn, cnt);
  if (!std::isfinite(orc_logmean(1.0, 1.0 + 1e-9))) g_bad = 1;
  const int bad[11] = {3, 0, 2, 0, 0, 1, 0, 0, 0, 0, 0};
  if (orc_create(bad, dcfg, affine.nE, affine.Ng, affine.X.data(), affine.nS, affine.se.data(), affine.sl.data(),
                 affine.so.data()) != nullptr)
    g_bad = 1;
  std::printf("oracle driver %s\n", g_bad ? "FAILED" : "ok");
  return g_bad;
}

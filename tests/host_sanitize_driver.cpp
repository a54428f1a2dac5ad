// Drives the host side of the C-ABI (context, mesh set-up and curl-form
// metrics, sizes, workspace planning, argument validation and error paths)
// without a GPU, for the AddressSanitizer / UndefinedBehaviorSanitizer build
// of the library's host code.  Exits non-zero on an unexpected status.
#include <cmath>
#include <cstdio>
#include <vector>

#include "dgx.h"

static int g_bad = 0;
static void expect(dg_status got, dg_status want, const char* what) {
  if (got != want) { std::fprintf(stderr, "%s: status %d, expected %d\n", what, (int)got, (int)want); g_bad = 1; }
}

struct Mesh {
  int nE, Ng, nS;
  std::vector<double> X;
  std::vector<int> se, sl, so;
};

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

static dg_config base(int N, int nodes, int form, int physics) {
  dg_config c{};
  c.N = N; c.nodes = nodes; c.volume_form = form; c.physics = physics;
  c.gamma = 1.4; c.mu = physics ? 0.01 : 0.0; c.Pr = 0.72; c.R = 1.0; c.Tref = 1.0; c.Ts = 0.4;
  return c;
}

int main() {
  const Mesh big = box(40, 40, 40, 1, 0.0), curved = box(3, 2, 2, 3, 0.1);
  const int cases[][4] = {{3, 0, 0, 0}, {7, 1, 1, 1}, {5, 1, 1, 1}, {3, 0, 1, 1}, {1, 1, 0, 0}, {2, 0, 0, 1}};
  for (const auto& k : cases) {
    dg_config cfg = base(k[0], k[1], k[2], k[3]);
    dg_ctx* ctx = nullptr;
    expect(dg_create(&cfg, &ctx), DG_OK, "dg_create");
    if (!ctx) continue;
    const Mesh& m = k[0] <= 3 ? big : curved;
    expect(dg_set_mesh(ctx, m.nE, m.Ng, m.X.data(), m.nS, m.se.data(), m.sl.data(), m.so.data()), DG_OK, "dg_set_mesh");
    int ne = 0, ns = 0, npe = 0;
    size_t len = 0;
    expect(dg_sizes(ctx, &ne, &ns, &npe, &len), DG_OK, "dg_sizes");
    std::vector<double> xyz((size_t)3 * ne * npe), Ja((size_t)9 * ne * npe), sJ((size_t)ne * npe),
        nv((size_t)3 * ns * (k[0] + 1) * (k[0] + 1));
    expect(dg_get_metrics(ctx, xyz.data(), Ja.data(), sJ.data(), nv.data()), DG_OK, "dg_get_metrics");
    expect(dg_node_coords(ctx, xyz.data()), DG_OK, "dg_node_coords");
    for (double v : sJ)
      if (!(v > 0.0) || !std::isfinite(v)) { g_bad = 1; break; }
    if (dg_workspace_bytes(ctx) == 0 || dg_workspace_bytes_adjoint(ctx) < dg_workspace_bytes(ctx)) g_bad = 1;
    // calls that need a device mesh or a workspace refuse
    double dummy[8];
    expect(dg_rhs(ctx, dummy, dummy + 4, 0.0, nullptr), DG_ERR_STATE, "dg_rhs without device mesh");
    expect(dg_bind_workspace(ctx, nullptr, 0), DG_ERR_ARG, "dg_bind_workspace(null)");
    expect(dg_profile(ctx, 0), DG_OK, "dg_profile off");
    long cnt = 0;
    double ms = 0;
    expect(dg_profile_query(ctx, "nonsense", &ms, &cnt), DG_ERR_ARG, "dg_profile_query unknown");
    expect(dg_destroy(ctx), DG_OK, "dg_destroy");
  }
  // invalid configurations and meshes
  dg_ctx* ctx = nullptr;
  dg_config bad = base(9, 1, 1, 1);
  expect(dg_create(&bad, &ctx), DG_ERR_UNSUPPORTED, "N out of range");
  bad = base(3, 1, 1, 1); bad.gamma = 1.0;
  expect(dg_create(&bad, &ctx), DG_ERR_ARG, "gamma");
  bad = base(3, 1, 7, 0);
  expect(dg_create(&bad, &ctx), DG_ERR_ARG, "form");
  expect(dg_create(nullptr, &ctx), DG_ERR_ARG, "null config");
  dg_config ok = base(2, 1, 0, 0);
  expect(dg_create(&ok, &ctx), DG_OK, "dg_create");
  Mesh m = box(2, 2, 1, 1, 0.0);
  std::vector<int> se = m.se;
  se[3] = 99;
  expect(dg_set_mesh(ctx, m.nE, m.Ng, m.X.data(), m.nS, se.data(), m.sl.data(), m.so.data()), DG_ERR_MESH, "bad side");
  std::vector<int> so = m.so;
  so[1] = 9;
  expect(dg_set_mesh(ctx, m.nE, m.Ng, m.X.data(), m.nS, m.se.data(), m.sl.data(), so.data()), DG_ERR_MESH, "orient");
  std::vector<double> X = m.X;
  for (size_t i = 0; i < X.size() / 3; ++i) X[i] = -X[i];   // mirrored x: negative Jacobian
  expect(dg_set_mesh(ctx, m.nE, m.Ng, X.data(), m.nS, m.se.data(), m.sl.data(), m.so.data()), DG_ERR_MESH, "folded");
  expect(dg_set_mesh(ctx, m.nE, m.Ng, m.X.data(), m.nS - 1, m.se.data(), m.sl.data(), m.so.data()), DG_ERR_MESH, "count");
  if (!dg_last_error(ctx) || !dg_last_error(ctx)[0]) g_bad = 1;
  expect(dg_destroy(ctx), DG_OK, "dg_destroy");
  double A[DG_RK_MAX_STAGES], B[DG_RK_MAX_STAGES], C[DG_RK_MAX_STAGES];
  int nst = 0;
  expect(dg_rk_coefficients(1, A, B, C, &nst), DG_OK, "rk coefficients");
  expect(dg_rk_coefficients(5, A, B, C, &nst), DG_ERR_ARG, "rk unknown");
  std::printf("host driver %s\n", g_bad ? "FAILED" : "ok");
  return g_bad;
}

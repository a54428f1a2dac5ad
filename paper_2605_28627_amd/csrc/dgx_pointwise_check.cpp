// dgx_pointwise_check.cpp -- host build of the library's point physics and its
// vector-Jacobian products, exported for the CPU test suite only (the product
// path runs these functions inside the HIP kernels).
#include "dgx_pointwise.hpp"

using namespace dgx;

static Phys make_phys(const double* c) {
  // c = {gamma, mu, Pr, R, riemann, twopoint, viscosity law, Tref, Ts}
  Phys P{};
  P.gamma = c[0]; P.gm1 = c[0] - 1.0; P.igm1 = 1.0 / (c[0] - 1.0); P.mu = c[1]; P.Pr = c[2]; P.R = c[3]; P.Rinv = 1.0 / c[3];
  P.lam = c[1] * c[0] * c[3] / ((c[0] - 1.0) * c[2]);
  P.kappa = c[0] * c[3] / ((c[0] - 1.0) * c[2]);
  P.riemann = (int)c[4]; P.twopoint = (int)c[5];
  P.visc_law = (int)c[6]; P.Tref = c[7]; P.Ts = c[8];
  return P;
}

extern "C" {

void pw_chandrashekar(const double* Ua, const double* Ub, const double* n, const double* c, double* F) {
  Phys P = make_phys(c);
  Aux a = make_aux(cons2prim(Ua, P.gm1)), b = make_aux(cons2prim(Ub, P.gm1));
  chandrashekar<double>(a, b, n, 0.5 / P.gm1, F);
}

void pw_chandrashekar_f32(const double* Ua, const double* Ub, const double* n, const double* c, double* F) {
  Phys P = make_phys(c);
  Aux a = make_aux(cons2prim(Ua, P.gm1)), b = make_aux(cons2prim(Ub, P.gm1));
  chandrashekar<float>(a, b, n, 0.5 / P.gm1, F);
}

// float flux about the reference state ref = (p0, ib0 = 2 p0 / rho0)
void pw_chandrashekar_f32_ref(const double* Ua, const double* Ub, const double* n, const double* c, const double* ref,
                              double* F) {
  Phys P = make_phys(c);
  Aux a = make_aux(cons2prim(Ua, P.gm1)), b = make_aux(cons2prim(Ub, P.gm1));
  chandrashekar<float>(a, b, n, 0.5 / P.gm1, F, ref[0], ref[1]);
}

void pw_euler_flux_f32_ref(const double* U, const double* n, const double* c, const double* ref, double* F) {
  Phys P = make_phys(c);
  euler_flux<float>(U, cons2prim(U, P.gm1), n, F, ref[0], P.gamma * ref[0] / P.gm1);
}

void pw_chandrashekar_vjp_a(const double* Ua, const double* Ub, const double* n, const double* c, const double* w,
                            double* Uab) {
  Phys P = make_phys(c);
  Prim qa = cons2prim(Ua, P.gm1);
  Aux a = make_aux(qa), b = make_aux(cons2prim(Ub, P.gm1));
  AuxBar ab;
  chandrashekar_vjp_a(a, b, n, 0.5 / P.gm1, w, ab);
  aux_vjp(qa, a, ab, P.gm1, Uab);
}

void pw_chandrashekar_vjp_ab(const double* Ua, const double* Ub, const double* n, const double* c, const double* w,
                             double* Uab, double* Ubb) {
  Phys P = make_phys(c);
  Prim qa = cons2prim(Ua, P.gm1), qb = cons2prim(Ub, P.gm1);
  Aux a = make_aux(qa), b = make_aux(qb);
  AuxBar aa, bb;
  chandrashekar_vjp_ab(a, b, n, 0.5 / P.gm1, w, aa, bb);
  aux_vjp(qa, a, aa, P.gm1, Uab);
  aux_vjp(qb, b, bb, P.gm1, Ubb);
}

void pw_entropy_vars(const double* U, const double* c, double* v) {
  Phys P = make_phys(c);
  entropy_vars(cons2prim(U, P.gm1), P.gm1, v);
}

void pw_entropy_to_cons(const double* v, const double* c, double* U) {
  Phys P = make_phys(c);
  entropy_to_cons(v, P.gm1, U);
}

void pw_entropy_vars_vjp(const double* U, const double* c, const double* Vb, double* Ub) {
  Phys P = make_phys(c);
  for (int k = 0; k < 5; ++k) Ub[k] = 0.0;
  entropy_vars_vjp(U, P.gm1, Vb, Ub);
}

void pw_entropy_to_cons_vjp(const double* v, const double* c, const double* Ub, double* Vb) {
  Phys P = make_phys(c);
  for (int k = 0; k < 5; ++k) Vb[k] = 0.0;
  entropy_to_cons_vjp(v, P.gm1, Ub, Vb);
}

void pw_euler_flux(const double* U, const double* n, const double* c, double* F) {
  Phys P = make_phys(c);
  euler_flux<double>(U, cons2prim(U, P.gm1), n, F);
}

void pw_euler_flux_vjp(const double* U, const double* n, const double* c, const double* w, double* Ub) {
  Phys P = make_phys(c);
  euler_flux_vjp(U, cons2prim(U, P.gm1), n, w, P.gm1, Ub);
}

void pw_viscous_flux(const double* U, const double* g, const double* n, const double* c, double* Gn) {
  Phys P = make_phys(c);
  viscous_flux<double>(cons2prim(U, P.gm1), g, P, n, Gn);
}

void pw_viscous_flux_vjp(const double* U, const double* g, const double* n, const double* c, const double* Gnb,
                         double* gb, double* Ub) {
  Phys P = make_phys(c);
  Prim q = cons2prim(U, P.gm1);
  double ub[3];
  viscous_flux_vjp(q, g, P, n, Gnb, gb, ub);
  prim_vjp(q, P.gm1, 0.0, ub, 0.0, Ub);
}

// d(sum_d sum_v M[d][v] G_d[1+v])/d(g, U) for the weights M[3][4] (row-major),
// with the viscosity law of c (constant or Sutherland).
void pw_viscous_tensor_vjp(const double* U, const double* g, const double* M, const double* c, double* gb,
                           double* Ub) {
  Phys P = make_phys(c);
  Prim q = cons2prim(U, P.gm1);
  double Mm[3][4], ub[3], rpb[2] = {0.0, 0.0};
  for (int d = 0; d < 3; ++d)
    for (int v = 0; v < 4; ++v) Mm[d][v] = M[4 * d + v];
  if (P.visc_law == 1)
    viscous_tensor_vjp<1>(q, g, P, Mm, gb, ub, rpb);
  else
    viscous_tensor_vjp<0>(q, g, P, Mm, gb, ub, rpb);
  prim_vjp(q, P.gm1, rpb[0], ub, rpb[1], Ub);
}

void pw_qvars(const double* U, const double* c, double* qv) {
  Phys P = make_phys(c);
  Prim q = cons2prim(U, P.gm1);
  qv[0] = q.u[0]; qv[1] = q.u[1]; qv[2] = q.u[2]; qv[3] = q.p / (q.rho * P.R);
}

void pw_qvars_vjp(const double* U, const double* c, const double* qb, double* Ub) {
  Phys P = make_phys(c);
  qvars_vjp(cons2prim(U, P.gm1), P.gm1, P.Rinv, qb, Ub);
}

// form 0 weak / 1 split; phys 0 Euler / 1 Navier-Stokes
void pw_surface_flux(int form, int phys, const double* UL, const double* UR, const double* gL, const double* gR,
                     const double* nh, double s, const double* c, double* Phi) {
  Phys P = make_phys(c);
  if (form == 0 && phys == 0) surface_flux<double, 0, 0>(UL, UR, gL, gR, nh, s, P, Phi);
  if (form == 0 && phys == 1) surface_flux<double, 0, 1>(UL, UR, gL, gR, nh, s, P, Phi);
  if (form == 1 && phys == 0) surface_flux<double, 1, 0>(UL, UR, gL, gR, nh, s, P, Phi);
  if (form == 1 && phys == 1) surface_flux<double, 1, 1>(UL, UR, gL, gR, nh, s, P, Phi);
}

void pw_surface_flux_vjp(int form, int phys, const double* UL, const double* UR, const double* gL, const double* gR,
                         const double* nh, double s, const double* c, const double* Phib, double* ULb, double* URb,
                         double* gLb, double* gRb) {
  Phys P = make_phys(c);
  if (form == 0 && phys == 0) surface_flux_vjp<0, 0>(UL, UR, gL, gR, nh, s, P, Phib, ULb, URb, gLb, gRb);
  if (form == 0 && phys == 1) surface_flux_vjp<0, 1>(UL, UR, gL, gR, nh, s, P, Phib, ULb, URb, gLb, gRb);
  if (form == 1 && phys == 0) surface_flux_vjp<1, 0>(UL, UR, gL, gR, nh, s, P, Phib, ULb, URb, gLb, gRb);
  if (form == 1 && phys == 1) surface_flux_vjp<1, 1>(UL, UR, gL, gR, nh, s, P, Phib, ULb, URb, gLb, gRb);
}

}  // extern "C"

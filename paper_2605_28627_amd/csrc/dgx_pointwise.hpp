// dgx_pointwise.hpp -- point physics of the DGSEM residual and its adjoint
// (host and device): conservative -> primitive, the advective, two-point,
// Rusanov and viscous fluxes, and their vector-Jacobian products.
//
// FT is the flux arithmetic type (double, or float in the FP32-flux mode);
// states, metrics and all accumulations are double.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "dgx_internal.hpp"

namespace dgx {

// ---------------------------------------------------------------------------
// Point physics.  FT is the flux arithmetic type (double, or float in the
// FP32-flux mode); states, metrics and all accumulations are double.
// ---------------------------------------------------------------------------
struct Prim {
  double rho, u[3], p;
};

__host__ __device__ inline Prim cons2prim(const double U[5], double gm1) {
  Prim q;
  q.rho = U[0];
  const double ri = 1.0 / U[0];
  q.u[0] = U[1] * ri; q.u[1] = U[2] * ri; q.u[2] = U[3] * ri;
  q.p = gm1 * (U[4] - 0.5 * q.rho * (q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2]));
  return q;
}

// Logarithmic mean (x - y)/(ln x - ln y) from precomputed logarithms; the
// atanh series (x+y)/(2 + u(2/3 + u(2/5 + u 2/7))), u = ((x-y)/(x+y))^2, below
// the threshold (1e-4 in double; 1e-2 in float where the truncation u^4/9 is
// below the float rounding).
template <typename FT>
__host__ __device__ inline FT log_mean(FT x, FT y, FT lx, FT ly) {
  const FT thr = sizeof(FT) == 8 ? FT(1e-4) : FT(1e-2);
  FT f = (x - y) / (x + y);
  FT u = f * f;
  if (u < thr) return (x + y) / (FT(2) + u * (FT(2.0 / 3.0) + u * (FT(2.0 / 5.0) + u * FT(2.0 / 7.0))));
  return (x - y) / (lx - ly);
}
// Reciprocal of the logarithmic mean.
template <typename FT>
__host__ __device__ inline FT inv_log_mean(FT x, FT y, FT lx, FT ly) {
  const FT thr = sizeof(FT) == 8 ? FT(1e-4) : FT(1e-2);
  FT f = (x - y) / (x + y);
  FT u = f * f;
  if (u < thr) return (FT(2) + u * (FT(2.0 / 3.0) + u * (FT(2.0 / 5.0) + u * FT(2.0 / 7.0)))) / (x + y);
  return (lx - ly) / (x - y);
}

// Reciprocal: hardware estimate refined by two Newton steps on the device
// (within an ulp of 1/x for the normal, finite x used here); exact division
// on the host.
__host__ __device__ inline double rcp_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
#else
  return 1.0 / x;
#endif
}
__host__ __device__ inline float rcp_nr(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
#else
  return 1.0f / x;
#endif
}

// 1/P(u) for P(u) = 2 + u(2/3 + u(2/5 + u 2/7)) in [2, 2+1e-4): Newton from 1/2.
template <typename FT>
__host__ __device__ inline FT inv_series(FT P) {
  FT r = FT(0.5);
  r = r * (FT(2) - P * r);
  r = r * (FT(2) - P * r);
  if (sizeof(FT) == 8) r = r * (FT(2) - P * r);
  return r;
}

// Per-node data a two-point flux needs from a partner node.
struct Aux {
  double rho, u[3], beta, lrho, lbeta, k;   // k = |u|^2
};

// Chandrashekar's kinetic-energy-preserving, entropy-conservative flux in the
// direction n (not normalised): F_rho = rho^ln {u}.n, F_m = p_hat n + {u} F_rho,
// F_E = F_rho (1/(2 (gamma-1) beta^ln) - {|u|^2}/2) + {u}.F_m.
// The log means are evaluated with two reciprocals per pair, 1/(rho_a+rho_b)
// and 1/(beta_a+beta_b) (the second also gives p_hat); the series branch
// divides by P(u) through inv_series, the direct branch needs one more.
//
// In float (the FP32-flux mode) p_hat and 1/beta^ln are formed as deviations
// from a reference state (p0, beta0 = 1/ib0), whose part is added in double:
//   p_hat - p0      = (1/2) ((rho_a - 2 p0 beta_a) + (rho_b - 2 p0 beta_b)) / (beta_a + beta_b),
//   1/beta^ln - ib0 = ((P - 2) - ((beta_a ib0 - 1) + (beta_b ib0 - 1))) / (beta_a + beta_b)
// (series branch, P the series), the bracketed sums in double, and rho^ln
// (series branch) as {rho} plus its float deviation -{rho} q/(1+q).  At low
// Mach numbers p and 1/beta are large and nearly constant, so float then
// rounds only their small deviations (the energy flux multiplies rho^ln by
// 1/beta^ln).  p0 = ib0 = 0 is no reference state.
template <typename FT>
__host__ __device__ inline void chandrashekar(const Aux& a, const Aux& b, const double n[3], double c1, double F[5],
                                              double p0 = 0.0, double ib0 = 0.0) {
  constexpr bool kRef = sizeof(FT) == 4;
  const FT thr = sizeof(FT) == 8 ? FT(1e-4) : FT(1e-2);
  const FT sr = FT(a.rho) + FT(b.rho), dr = FT(a.rho) - FT(b.rho);
  const FT sb = FT(a.beta) + FT(b.beta), db = FT(a.beta) - FT(b.beta);
  const FT rsr = rcp_nr(sr), rsb = rcp_nr(sb);
  const FT fr = dr * rsr, ur = fr * fr;
  const FT fb = db * rsb, ub2 = fb * fb;
  FT rho_ln, ibeta_ln;   // (kRef: 1/beta^ln - ib0)
  double rho_lnd;        // rho^ln in double
  if (ur < thr) {
    if constexpr (kRef) {
      // rho^ln = {rho} / (1 + q), q = (P - 2)/2: the deviation -{rho} q/(1+q)
      // in float (1/(1+q) = 1 - q + q^2 to float accuracy for q < 0.0034)
      const FT q = ur * (FT(1.0 / 3.0) + ur * (FT(1.0 / 5.0) + ur * FT(1.0 / 7.0)));
      rho_ln = -FT(0.5) * sr * q * (FT(1) - q + q * q);
      rho_lnd = 0.5 * (a.rho + b.rho) + double(rho_ln);
    } else {
      const FT P = FT(2) + ur * (FT(2.0 / 3.0) + ur * (FT(2.0 / 5.0) + ur * FT(2.0 / 7.0)));
      rho_ln = sr * inv_series<FT>(P);
      rho_lnd = double(rho_ln);
    }
  } else {
    rho_ln = dr * rcp_nr(FT(a.lrho) - FT(b.lrho));
    rho_lnd = double(rho_ln);
  }
  if (ub2 < thr) {
    if constexpr (kRef) {
      const FT Pm2 = ub2 * (FT(2.0 / 3.0) + ub2 * (FT(2.0 / 5.0) + ub2 * FT(2.0 / 7.0)));
      const FT dsb = FT((a.beta * ib0 - 1.0) + (b.beta * ib0 - 1.0));
      ibeta_ln = (Pm2 - dsb) * rsb;
    } else {
      ibeta_ln = (FT(2) + ub2 * (FT(2.0 / 3.0) + ub2 * (FT(2.0 / 5.0) + ub2 * FT(2.0 / 7.0)))) * rsb;
    }
  } else {
    ibeta_ln = (FT(a.lbeta) - FT(b.lbeta)) * rcp_nr(db);
    if constexpr (kRef) ibeta_ln -= FT(ib0);
  }
  FT phat;
  if constexpr (kRef)
    phat = FT(0.5) * FT((a.rho - 2.0 * p0 * a.beta) + (b.rho - 2.0 * p0 * b.beta)) * rsb;
  else
    phat = FT(0.5) * sr * rsb;
  const FT X = ibeta_ln * FT(c1) - FT(0.25) * (FT(a.k) + FT(b.k));
  const double um0 = 0.5 * (a.u[0] + b.u[0]), um1 = 0.5 * (a.u[1] + b.u[1]), um2 = 0.5 * (a.u[2] + b.u[2]);
  const double umn = um0 * n[0] + um1 * n[1] + um2 * n[2];
  const double Fr = rho_lnd * umn;
  const double ph = kRef ? double(phat) + p0 : double(phat);
  const double Xd = kRef ? double(X) + c1 * ib0 : double(X);
  F[0] = Fr;
  F[1] = ph * n[0] + um0 * Fr;
  F[2] = ph * n[1] + um1 * Fr;
  F[3] = ph * n[2] + um2 * Fr;
  F[4] = Fr * Xd + (um0 * F[1] + um1 * F[2] + um2 * F[3]);
}

// Two-point record with the logarithms supplied (ln rho, ln beta).
__host__ __device__ inline Aux make_aux_logs(const Prim& q, double lrho, double lbeta) {
  Aux a;
  a.rho = q.rho; a.u[0] = q.u[0]; a.u[1] = q.u[1]; a.u[2] = q.u[2];
  a.beta = 0.5 * q.rho / q.p;
  a.lrho = lrho;
  a.lbeta = lbeta;
  a.k = q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2];
  return a;
}

__host__ __device__ inline Aux make_aux(const Prim& q) {
  Aux a;
  a.rho = q.rho; a.u[0] = q.u[0]; a.u[1] = q.u[1]; a.u[2] = q.u[2];
  a.beta = 0.5 * q.rho / q.p;
  a.lrho = log(q.rho);
  a.lbeta = log(a.beta);
  a.k = q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2];
  return a;
}

// Entropy variables of the entropy S = -rho s/(gamma-1), s = ln p - gamma ln rho,
// that the Chandrashekar flux conserves: with b = rho/p,
//   v = ((gamma - s)/(gamma-1) - b |u|^2/2,  b u,  -b).
__host__ __device__ inline void entropy_vars(const Prim& q, double gm1, double v[5]) {
  const double b = q.rho / q.p;
  const double s = log(q.p) - (gm1 + 1.0) * log(q.rho);
  v[0] = (gm1 + 1.0 - s) / gm1 - 0.5 * b * (q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2]);
  v[1] = b * q.u[0]; v[2] = b * q.u[1]; v[3] = b * q.u[2];
  v[4] = -b;
}
// Conservative state of the entropy variables v: b = -v_4, u = v_{1..3}/b and,
// with z = v_0 + b |u|^2/2 = (gamma - s)/(gamma-1), ln rho = z - (gamma + ln b)/(gamma-1).
// logs (optional) receives ln rho and ln beta = ln(b/2) (beta = rho/(2p)), the
// two logarithms a two-point record needs, as by-products.
__host__ __device__ inline void entropy_to_cons(const double v[5], double gm1, double U[5], double* logs = nullptr) {
  const double b = -v[4];
  const double ib = 1.0 / b;
  const double u0 = v[1] * ib, u1 = v[2] * ib, u2 = v[3] * ib;
  const double k = u0 * u0 + u1 * u1 + u2 * u2;
  const double z = v[0] + 0.5 * b * k;
  const double lb = log(b);
  const double lrho = z - (gm1 + 1.0 + lb) / gm1;
  const double rho = exp(lrho);
  if (logs) { logs[0] = lrho; logs[1] = lb - 0.69314718055994530942; }
  U[0] = rho;
  U[1] = rho * u0; U[2] = rho * u1; U[3] = rho * u2;
  U[4] = rho * ib / gm1 + 0.5 * rho * k;
}

// Advective flux in direction n of the state described by a two-point record
// (rho, u, beta = rho/(2p), |u|^2).
template <typename FT>
__host__ __device__ inline void aux_flux(const Aux& a, double gm1, const double n[3], double F[5]) {
  const double p = 0.5 * a.rho / a.beta;
  const double un = a.u[0] * n[0] + a.u[1] * n[1] + a.u[2] * n[2];
  const double H = p / gm1 + 0.5 * a.rho * a.k + p;
  F[0] = a.rho * un;
  F[1] = a.rho * a.u[0] * un + p * n[0];
  F[2] = a.rho * a.u[1] * un + p * n[1];
  F[3] = a.rho * a.u[2] * un + p * n[2];
  F[4] = H * un;
}

// Advective flux of U in direction n (not normalised).  In float the pressure
// and the total enthalpy enter as deviations p - p0, H - h0 from a reference
// state (h0 = gamma p0 / (gamma - 1)), whose part is added in double.
template <typename FT>
__host__ __device__ inline void euler_flux(const double U[5], const Prim& q, const double n[3], double F[5],
                                           double p0 = 0.0, double h0 = 0.0) {
  if constexpr (sizeof(FT) == 8) {
    const double un = q.u[0] * n[0] + q.u[1] * n[1] + q.u[2] * n[2];
    F[0] = U[0] * un;
    F[1] = U[1] * un + q.p * n[0];
    F[2] = U[2] * un + q.p * n[1];
    F[3] = U[3] * un + q.p * n[2];
    F[4] = (U[4] + q.p) * un;
  } else {
    // Cartesian flux components in float, contraction with the metric in double.
    const float r = float(q.rho), u0 = float(q.u[0]), u1 = float(q.u[1]), u2 = float(q.u[2]), p = float(q.p - p0);
    const float H = float((U[4] + q.p) - h0);
    const float uu[3] = {u0, u1, u2};
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float ud = uu[d];
      const float ru = r * ud;
      acc[0] += n[d] * double(ru);
      acc[1] += n[d] * double(ru * u0 + (d == 0 ? p : 0.0f));
      acc[2] += n[d] * double(ru * u1 + (d == 1 ? p : 0.0f));
      acc[3] += n[d] * double(ru * u2 + (d == 2 ? p : 0.0f));
      acc[4] += n[d] * double(H * ud);
    }
    const double un = q.u[0] * n[0] + q.u[1] * n[1] + q.u[2] * n[2];
    acc[1] += p0 * n[0]; acc[2] += p0 * n[1]; acc[3] += p0 * n[2];
    acc[4] += h0 * un;
    for (int v = 0; v < 5; ++v) F[v] = acc[v];
  }
}

// Dynamic viscosity at the node's temperature T = p/(rho R): constant, or
// Sutherland's law mu (T/Tref)^(3/2) (1 + Ts) / (T/Tref + Ts).
template <typename FT>
__host__ __device__ inline FT visc_mu(const Prim& q, const Phys& P) {
  if (P.visc_law == 0) return FT(P.mu);
  const FT th = FT(q.p * P.Rinv / (q.rho * P.Tref));
  return FT(P.mu) * th * sqrt(th) * FT(1.0 + P.Ts) / (th + FT(P.Ts));
}

// Viscous flux G_d (d = 0..2) for the momentum and energy components (v = 1..4),
// contracted with n: Gn[v-1] = sum_d n_d G_d[v].  g[3a+d] = dq_a/dx_d, q = (u,v,w,T).
// VL: the viscosity law at compile time (0 constant, 1 Sutherland), or -1 to
// follow P.visc_law at run time.
template <typename FT, int VL = -1>
__host__ __device__ inline void viscous_flux(const Prim& q, const double g[12], const Phys& P, const double n[3],
                                             double Gn[4]) {
  const bool suth = VL == 1 || (VL == -1 && P.visc_law == 1);
  const FT mu = suth ? visc_mu<FT>(q, P) : FT(P.mu);
  const FT lam = suth ? mu * FT(P.kappa) : FT(P.lam);
  FT gg[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) gg[c] = FT(g[c]);
  const FT divu = gg[0] + gg[4] + gg[8];
  FT tau[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d) tau[a][d] = mu * (gg[3 * a + d] + gg[3 * d + a]);
  const FT t2 = FT(2.0 / 3.0) * mu * divu;
  tau[0][0] -= t2; tau[1][1] -= t2; tau[2][2] -= t2;
  const FT u0 = FT(q.u[0]), u1 = FT(q.u[1]), u2 = FT(q.u[2]);
  double acc[4] = {0, 0, 0, 0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    acc[0] += n[d] * double(tau[0][d]);
    acc[1] += n[d] * double(tau[1][d]);
    acc[2] += n[d] * double(tau[2][d]);
    acc[3] += n[d] * double(tau[d][0] * u0 + tau[d][1] * u1 + tau[d][2] * u2 + lam * gg[9 + d]);
  }
  Gn[0] = acc[0]; Gn[1] = acc[1]; Gn[2] = acc[2]; Gn[3] = acc[3];
}

// Roe's dissipation |A~|(UR - UL) on the unit normal nh (Roe 1981): Roe
// averages (weights sqrt(rho)), wave strengths of the two acoustic, the
// entropy and the two shear waves, with the Harten & Hyman (1983) entropy fix
// on the acoustic speeds: delta = max(0, l~ - l(UL), l(UR) - l~), and where
// |l~| < delta the speed (l~^2 + delta^2) / (2 delta).  FT arithmetic.
// Dual numbers (value, derivative along one direction) for the adjoint of
// Roe's dissipation: its Jacobian is taken column by column in forward mode,
// through the same roe_core as the residual (kinks on the forward's branch).
struct Dual {
  double v, d;
  __host__ __device__ Dual() : v(0.0), d(0.0) {}
  __host__ __device__ explicit Dual(double x, double dx = 0.0) : v(x), d(dx) {}
  // (found by argument-dependent lookup only, so that double arithmetic
  // elsewhere in this namespace keeps ::sqrt and ::fabs)
  friend __host__ __device__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
  friend __host__ __device__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
  friend __host__ __device__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
  friend __host__ __device__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
  friend __host__ __device__ Dual operator/(Dual a, Dual b) {
    const double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
  }
  friend __host__ __device__ Dual sqrt(Dual a) {
    const double r = ::sqrt(a.v);
    return Dual(r, 0.5 * a.d / r);
  }
  friend __host__ __device__ Dual fabs(Dual a) { return a.v < 0.0 ? -a : a; }
  friend __host__ __device__ Dual log(Dual a) { return Dual(::log(a.v), a.d / a.v); }
  friend __host__ __device__ Dual exp(Dual a) {
    const double e = ::exp(a.v);
    return Dual(e, e * a.d);
  }
  friend __host__ __device__ Dual operator*(double s, Dual a) { return Dual(s * a.v, s * a.d); }
  friend __host__ __device__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
  friend __host__ __device__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
};

template <typename FT>
__host__ __device__ inline FT hh_speed(FT lm, FT lL, FT lR) {
  const FT a = fabs(lm);
  FT delta = lm - lL > lR - lm ? lm - lL : lR - lm;
  delta = delta > FT(0) ? delta : FT(0);
  return a < delta ? (lm * lm + delta * delta) / (FT(2) * delta) : a;
}
// The dissipation itself on primitive inputs in T arithmetic: T = FT for the
// residual, or the dual numbers of its adjoint (Dual below); EL, ER the total
// energies.
template <typename T>
__host__ __device__ inline void roe_core(const T& EL, const T& ER, const T& rl, const T& rr, const T ul[3],
                                         const T ur[3], const T& pl, const T& pr, const T n[3], const T& gam, T D[5]) {
  const T sl = sqrt(rl), sr = sqrt(rr);
  const T iw = T(1) / (sl + sr);
  const T HL = (EL + pl) / rl, HR = (ER + pr) / rr;
  T um[3], du[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    um[d] = (sl * ul[d] + sr * ur[d]) * iw;
    du[d] = ur[d] - ul[d];
  }
  const T Hm = (sl * HL + sr * HR) * iw;
  const T q2 = um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
  const T c2 = (gam - T(1)) * (Hm - T(0.5) * q2);
  const T cm = sqrt(c2), ic2 = T(1) / c2;
  const T rm = sl * sr;
  const T unm = um[0] * n[0] + um[1] * n[1] + um[2] * n[2];
  const T dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  const T dp = pr - pl;
  const T a1 = T(0.5) * (dp - rm * cm * dun) * ic2;
  const T a5 = T(0.5) * (dp + rm * cm * dun) * ic2;
  const T a2 = (rr - rl) - dp * ic2;
  const T cl = sqrt(gam * pl / rl), cr = sqrt(gam * pr / rr);
  const T unl = ul[0] * n[0] + ul[1] * n[1] + ul[2] * n[2];
  const T unr = ur[0] * n[0] + ur[1] * n[1] + ur[2] * n[2];
  const T w1 = hh_speed<T>(unm - cm, unl - cl, unr - cr) * a1;
  const T w5 = hh_speed<T>(unm + cm, unl + cl, unr + cr) * a5;
  const T l2 = fabs(unm);
  const T w2 = l2 * a2, wsh = l2 * rm;
  const T udu = um[0] * du[0] + um[1] * du[1] + um[2] * du[2];
  D[0] = w1 + w2 + w5;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    D[1 + d] = w1 * (um[d] - cm * n[d]) + w2 * um[d] + wsh * (du[d] - dun * n[d]) + w5 * (um[d] + cm * n[d]);
  D[4] = w1 * (Hm - unm * cm) + w2 * T(0.5) * q2 + wsh * (udu - unm * dun) + w5 * (Hm + unm * cm);
}
template <typename FT>
__host__ __device__ inline void roe_dissipation(const double UL[5], const double UR[5], const Prim& qL, const Prim& qR,
                                                const double nh[3], const Phys& P, double D[5]) {
  const FT gam = FT(P.gamma);
  const FT n[3] = {FT(nh[0]), FT(nh[1]), FT(nh[2])};
  const FT rl = FT(qL.rho), rr = FT(qR.rho), pl = FT(qL.p), pr = FT(qR.p);
  const FT ul[3] = {FT(qL.u[0]), FT(qL.u[1]), FT(qL.u[2])}, ur[3] = {FT(qR.u[0]), FT(qR.u[1]), FT(qR.u[2])};
  FT Df[5];
  roe_core<FT>(FT(UL[4]), FT(UR[4]), rl, rr, ul, ur, pl, pr, n, gam, Df);
#pragma unroll
  for (int v = 0; v < 5; ++v) D[v] = double(Df[v]);
}

// Advective part of the outward (master) surface flux at one face node:
// Phi = [F*(UL,UR).n - lambda_max/2 (UR-UL)] s.
// ROE selects Roe's dissipation at compile time (its temporaries would raise
// the register count of every kernel as a run-time branch); otherwise
// P.riemann chooses Rusanov or no dissipation.  Split form: logs (optional)
// supplies ln rho, ln beta of UL then UR; with aux the two-point record of UR
// (side 1) or of UL (side 0) is returned in *aux.
template <typename FT, int FORM, int ROE = 0>
__host__ __device__ inline void surface_flux_adv(const double UL[5], const double UR[5], const double nh[3], double s,
                                                 const Phys& P, double Phi[5], Aux* aux = nullptr, int side = 0,
                                                 const double* logs = nullptr) {
  const Prim qL = cons2prim(UL, P.gm1), qR = cons2prim(UR, P.gm1);
  const double nv[3] = {nh[0] * s, nh[1] * s, nh[2] * s};
  if (FORM == 1 && P.twopoint == 0) {
    const Aux aL = logs ? make_aux_logs(qL, logs[0], logs[1]) : make_aux(qL);
    const Aux aR = logs ? make_aux_logs(qR, logs[2], logs[3]) : make_aux(qR);
    chandrashekar<FT>(aL, aR, nv, 0.5 / P.gm1, Phi, P.p0, P.ib0);
    if (aux) *aux = side ? aR : aL;
  } else {
    if (FORM == 1 && aux) *aux = make_aux(side ? qR : qL);
    double FL[5], FR[5];
    euler_flux<FT>(UL, qL, nv, FL, P.p0, P.h0);
    euler_flux<FT>(UR, qR, nv, FR, P.p0, P.h0);
#pragma unroll
    for (int v = 0; v < 5; ++v) Phi[v] = 0.5 * (FL[v] + FR[v]);
  }
  if constexpr (ROE == 1) {
    double D[5];
    roe_dissipation<FT>(UL, UR, qL, qR, nh, P, D);
    const double hs = 0.5 * s;
#pragma unroll
    for (int v = 0; v < 5; ++v) Phi[v] -= hs * D[v];
  } else if (P.riemann == 0) {
    const FT cL = sqrt(FT(P.gamma) * FT(qL.p) / FT(qL.rho));
    const FT cR = sqrt(FT(P.gamma) * FT(qR.p) / FT(qR.rho));
    const FT unL = FT(qL.u[0] * nh[0] + qL.u[1] * nh[1] + qL.u[2] * nh[2]);
    const FT unR = FT(qR.u[0] * nh[0] + qR.u[1] * nh[1] + qR.u[2] * nh[2]);
    const FT lL = fabs(unL) + cL, lR = fabs(unR) + cR;
    const double lmax = double(lL >= lR ? lL : lR);
    const double hs = 0.5 * (lmax * s);
#pragma unroll
    for (int v = 0; v < 5; ++v) Phi[v] -= hs * (UR[v] - UL[v]);
  }
}

// Outward (master) surface flux at one face node:
// Phi = [F*(UL,UR).n - lambda_max/2 (UR-UL)] s - 1/2 (G(UL,gL) + G(UR,gR)).n s
template <typename FT, int FORM, int PHYS>
__host__ __device__ inline void surface_flux(const double UL[5], const double UR[5], const double* gL,
                                             const double* gR, const double nh[3], double s, const Phys& P,
                                             double Phi[5]) {
  if (P.riemann == 2)
    surface_flux_adv<FT, FORM, 1>(UL, UR, nh, s, P, Phi);
  else
    surface_flux_adv<FT, FORM, 0>(UL, UR, nh, s, P, Phi);
  if constexpr (PHYS == 1) {
    const double nv[3] = {nh[0] * s, nh[1] * s, nh[2] * s};
    double GL[4], GR[4];
    viscous_flux<FT>(cons2prim(UL, P.gm1), gL, P, nv, GL);
    viscous_flux<FT>(cons2prim(UR, P.gm1), gR, P, nv, GR);
#pragma unroll
    for (int v = 0; v < 4; ++v) Phi[1 + v] -= 0.5 * (GL[v] + GR[v]);
  }
}

// ---------------------------------------------------------------------------
// Vector-Jacobian products (reverse mode, FP64).  Each function returns
// (d(w . f)/d input) for the forward function f of the same name above, with
// the branch taken by the forward evaluation (log-mean series/direct, the
// larger Rusanov wave speed, the sign of u.n with +1 at 0).
// ---------------------------------------------------------------------------

// (rho, u, p) -> U: adjoints rb, ub[3], pb of the primitive variables.
__host__ __device__ inline void prim_vjp(const Prim& q, double gm1, double rb, const double ub[3], double pb,
                                         double Ub[5]) {
  const double ri = 1.0 / q.rho;
  const double k = q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2];
  Ub[4] = gm1 * pb;
  Ub[1] = ub[0] * ri - gm1 * pb * q.u[0];
  Ub[2] = ub[1] * ri - gm1 * pb * q.u[1];
  Ub[3] = ub[2] * ri - gm1 * pb * q.u[2];
  Ub[0] = rb - (ub[0] * q.u[0] + ub[1] * q.u[1] + ub[2] * q.u[2]) * ri + 0.5 * gm1 * pb * k;
}

// Adjoints of the entropy projection of the split form on Gauss nodes
// (u~ = u(E v(U))), by forward-mode columns of the two maps: Vb += (du/dv)^T Ub
// at the entropy variables v, and Ub += (dv/dU)^T Vb at the state U.
__host__ __device__ inline void entropy_to_cons_vjp(const double v[5], double gm1, const double Ub[5], double Vb[5]) {
#pragma unroll 1
  for (int k = 0; k < 5; ++k) {
    Dual x[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) x[c] = Dual(v[c], c == k ? 1.0 : 0.0);
    const Dual b = -x[4];
    const Dual ib = Dual(1.0) / b;
    const Dual u0 = x[1] * ib, u1 = x[2] * ib, u2 = x[3] * ib;
    const Dual kk = u0 * u0 + u1 * u1 + u2 * u2;
    const Dual z = x[0] + 0.5 * (b * kk);
    const Dual rho = exp(z - (Dual(gm1 + 1.0) + log(b)) / Dual(gm1));
    const Dual U[5] = {rho, rho * u0, rho * u1, rho * u2, rho * ib / Dual(gm1) + 0.5 * (rho * kk)};
    double sdot = 0.0;
#pragma unroll
    for (int c = 0; c < 5; ++c) sdot += Ub[c] * U[c].d;
#pragma unroll
    for (int c = 0; c < 5; ++c) Vb[c] += c == k ? sdot : 0.0;
  }
}
__host__ __device__ inline void entropy_vars_vjp(const double Uin[5], double gm1, const double Vb[5], double Ub[5]) {
#pragma unroll 1
  for (int k = 0; k < 5; ++k) {
    Dual x[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) x[c] = Dual(Uin[c], c == k ? 1.0 : 0.0);
    const Dual ri = Dual(1.0) / x[0];
    const Dual u0 = x[1] * ri, u1 = x[2] * ri, u2 = x[3] * ri;
    const Dual kk = u0 * u0 + u1 * u1 + u2 * u2;
    const Dual p = Dual(gm1) * (x[4] - 0.5 * (x[0] * kk));
    const Dual b = x[0] / p;
    const Dual s = log(p) - Dual(gm1 + 1.0) * log(x[0]);
    const Dual v[5] = {(Dual(gm1 + 1.0) - s) / Dual(gm1) - 0.5 * (b * kk), b * u0, b * u1, b * u2, -b};
    double sdot = 0.0;
#pragma unroll
    for (int c = 0; c < 5; ++c) sdot += Vb[c] * v[c].d;
#pragma unroll
    for (int c = 0; c < 5; ++c) Ub[c] += c == k ? sdot : 0.0;
  }
}

// Adjoint of Roe's dissipation D(UL, UR) on the unit normal nh: ULb, URb +=
// (dD/dU)^T Db, one forward-mode column per entry of UL and UR (primitives by
// the operations of cons2prim).
__host__ __device__ inline void roe_dissipation_vjp(const double UL[5], const double UR[5], const double nh[3],
                                                    const Phys& P, const double Db[5], double ULb[5], double URb[5]) {
  const Dual gam(P.gamma);
  const Dual n[3] = {Dual(nh[0]), Dual(nh[1]), Dual(nh[2])};
#pragma unroll 1
  for (int k = 0; k < 10; ++k) {
    Dual uL[5], uR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      uL[v] = Dual(UL[v], k == v ? 1.0 : 0.0);
      uR[v] = Dual(UR[v], k == 5 + v ? 1.0 : 0.0);
    }
    const Dual riL = Dual(1.0) / uL[0], riR = Dual(1.0) / uR[0];
    const Dual ul[3] = {uL[1] * riL, uL[2] * riL, uL[3] * riL}, ur[3] = {uR[1] * riR, uR[2] * riR, uR[3] * riR};
    const Dual gm1(P.gm1);
    const Dual pl = gm1 * (uL[4] - Dual(0.5) * uL[0] * (ul[0] * ul[0] + ul[1] * ul[1] + ul[2] * ul[2]));
    const Dual pr = gm1 * (uR[4] - Dual(0.5) * uR[0] * (ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]));
    Dual D[5];
    roe_core<Dual>(uL[4], uR[4], uL[0], uR[0], ul, ur, pl, pr, n, gam, D);
    double sdot = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) sdot += Db[v] * D[v].d;
    // (selects, not a run-time index, keep ULb and URb in registers)
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      ULb[v] += k == v ? sdot : 0.0;
      URb[v] += k == 5 + v ? sdot : 0.0;
    }
  }
}

// Adjoint of the lifted variables q = (u, v, w, T = p/(rho R)).
__host__ __device__ inline void qvars_vjp(const Prim& q, double gm1, double Rinv, const double qb[4], double Ub[5]) {
  const double ri = 1.0 / q.rho;
  const double T = q.p * ri * Rinv;
  const double pb = qb[3] * ri * Rinv;
  const double rb = -qb[3] * T * ri;
  prim_vjp(q, gm1, rb, qb, pb, Ub);
}

// Adjoint of Aux = (rho, u, beta = rho/(2p), ln rho, ln beta, |u|^2).
struct AuxBar {
  double rho, u[3], beta, lrho, lbeta, k;
};

__host__ __device__ inline void aux_vjp(const Prim& q, const Aux& a, const AuxBar& b, double gm1, double Ub[5]) {
  const double betab = b.beta + b.lbeta / a.beta;
  double rb = b.rho + b.lrho / a.rho + betab * 0.5 / q.p;
  const double pb = -betab * a.beta / q.p;
  const double ub[3] = {b.u[0] + 2.0 * q.u[0] * b.k, b.u[1] + 2.0 * q.u[1] * b.k, b.u[2] + 2.0 * q.u[2] * b.k};
  prim_vjp(q, gm1, rb, ub, pb, Ub);
}

// The logarithmic mean L(x, y; lx, ly) and its partial derivatives, from the
// sum s = x + y and is = 1/s (branch as in the forward; reciprocals by rcp_nr):
//   series (u = ((x-y)/s)^2 < 1e-4): L = s/P(u), dL/dx = 1/P - c y, dL/dy = 1/P + c x,
//     c = 4 f P'(u) / (P^2 s), f = (x-y)/s;
//   direct: L = (x-y)/(lx-ly), dL/dx = -dL/dy = 1/(lx-ly), dL/dlx = -dL/dly = -L/(lx-ly).
__host__ __device__ inline void log_mean_d(double x, double y, double lx, double ly, double s, double is, double& L,
                                           double& dx, double& dy, double& dlx, double& dly) {
  const double f = (x - y) * is, u = f * f;
  if (u < 1e-4) {
    const double P = 2.0 + u * (2.0 / 3.0 + u * (2.0 / 5.0 + u * (2.0 / 7.0)));
    const double dP = 2.0 / 3.0 + u * (4.0 / 5.0 + u * (6.0 / 7.0));
    const double iP = rcp_nr(P);
    L = s * iP;
    const double c = 4.0 * f * dP * iP * iP * is;
    dx = iP - c * y;
    dy = iP + c * x;
    dlx = 0.0;
    dly = 0.0;
  } else {
    const double idl = rcp_nr(lx - ly);
    L = (x - y) * idl;
    const double q = L * idl;
    dx = idl;
    dy = -idl;
    dlx = -q;
    dly = q;
  }
}
// The reciprocal logarithmic mean I = 1/L and its partial derivatives:
//   series: I = P/s, dI/dx = -P/s^2 + c y, dI/dy = -P/s^2 - c x, c = 4 f P'(u)/s^3;
//   direct: I = (lx-ly)/(x-y), dI/dx = -dI/dy = -I/(x-y), dI/dlx = -dI/dly = 1/(x-y).
__host__ __device__ inline void inv_log_mean_d(double x, double y, double lx, double ly, double s, double is,
                                               double& I, double& dx, double& dy, double& dlx, double& dly) {
  const double f = (x - y) * is, u = f * f;
  if (u < 1e-4) {
    const double P = 2.0 + u * (2.0 / 3.0 + u * (2.0 / 5.0 + u * (2.0 / 7.0)));
    const double dP = 2.0 / 3.0 + u * (4.0 / 5.0 + u * (6.0 / 7.0));
    I = P * is;
    const double c = 4.0 * f * dP * is * is * is;
    const double base = -I * is;
    dx = base + c * y;
    dy = base - c * x;
    dlx = 0.0;
    dly = 0.0;
  } else {
    const double id = rcp_nr(x - y);
    I = (lx - ly) * id;
    const double q = I * id;
    dx = -q;
    dy = q;
    dlx = id;
    dly = -id;
  }
}

// d(w . F#(a, b; n))/d aux_a and d aux_b for Chandrashekar's flux in one
// reverse sweep (FP64 forward).  The averages are symmetric, so the two
// argument adjoints share every term except the log-mean derivatives; three
// reciprocals (1/(rho_a+rho_b), 1/(beta_a+beta_b), and the log mean's own)
// serve the whole sweep.
__host__ __device__ inline void chandrashekar_vjp_ab(const Aux& a, const Aux& b, const double n[3], double c1,
                                                     const double w[5], AuxBar& aa, AuxBar& bb) {
  const double sr = a.rho + b.rho, isr = rcp_nr(sr);
  const double S = a.beta + b.beta, iS = rcp_nr(S);
  double rho_ln, rdx, rdy, rdlx, rdly, ibl, bdx, bdy, bdlx, bdly;
  log_mean_d(a.rho, b.rho, a.lrho, b.lrho, sr, isr, rho_ln, rdx, rdy, rdlx, rdly);
  inv_log_mean_d(a.beta, b.beta, a.lbeta, b.lbeta, S, iS, ibl, bdx, bdy, bdlx, bdly);
  const double phat = 0.5 * sr * iS;
  const double X = ibl * c1 - 0.25 * (a.k + b.k);
  const double um[3] = {0.5 * (a.u[0] + b.u[0]), 0.5 * (a.u[1] + b.u[1]), 0.5 * (a.u[2] + b.u[2])};
  const double umn = um[0] * n[0] + um[1] * n[1] + um[2] * n[2];
  const double Fr = rho_ln * umn;
  // reverse sweep
  double Fmb[3];
  for (int d = 0; d < 3; ++d) Fmb[d] = w[1 + d] + w[4] * um[d];
  const double Frb = w[0] + w[4] * X + (Fmb[0] * um[0] + Fmb[1] * um[1] + Fmb[2] * um[2]);
  const double Xb = w[4] * Fr;
  const double phatb = Fmb[0] * n[0] + Fmb[1] * n[1] + Fmb[2] * n[2];
  const double rlnb = Frb * umn;
  const double umnb = Frb * rho_ln;
  for (int d = 0; d < 3; ++d) {
    const double Fm = phat * n[d] + um[d] * Fr;
    const double umb = w[4] * Fm + Fmb[d] * Fr + umnb * n[d];
    aa.u[d] = bb.u[d] = 0.5 * umb;
  }
  const double iblb = c1 * Xb;
  aa.k = bb.k = -0.25 * Xb;
  const double rho_p = 0.5 * phatb * iS, beta_p = -phatb * phat * iS;
  aa.rho = rho_p + rlnb * rdx;
  bb.rho = rho_p + rlnb * rdy;
  aa.lrho = rlnb * rdlx;
  bb.lrho = rlnb * rdly;
  aa.beta = beta_p + iblb * bdx;
  bb.beta = beta_p + iblb * bdy;
  aa.lbeta = iblb * bdlx;
  bb.lbeta = iblb * bdly;
}

// d(w . F#(a, b; n))/d aux_a for Chandrashekar's flux (FP64 forward).
__host__ __device__ inline void chandrashekar_vjp_a(const Aux& a, const Aux& b, const double n[3], double c1,
                                                    const double w[5], AuxBar& ab) {
  const double sr = a.rho + b.rho, isr = rcp_nr(sr);
  const double S = a.beta + b.beta, iS = rcp_nr(S);
  double rho_ln, rdx, rdy, rdlx, rdly, ibl, bdx, bdy, bdlx, bdly;
  log_mean_d(a.rho, b.rho, a.lrho, b.lrho, sr, isr, rho_ln, rdx, rdy, rdlx, rdly);
  inv_log_mean_d(a.beta, b.beta, a.lbeta, b.lbeta, S, iS, ibl, bdx, bdy, bdlx, bdly);
  const double phat = 0.5 * sr * iS;
  const double X = ibl * c1 - 0.25 * (a.k + b.k);
  const double um[3] = {0.5 * (a.u[0] + b.u[0]), 0.5 * (a.u[1] + b.u[1]), 0.5 * (a.u[2] + b.u[2])};
  const double umn = um[0] * n[0] + um[1] * n[1] + um[2] * n[2];
  const double Fr = rho_ln * umn;
  // reverse sweep
  double Fmb[3];
  for (int d = 0; d < 3; ++d) Fmb[d] = w[1 + d] + w[4] * um[d];
  const double Frb = w[0] + w[4] * X + (Fmb[0] * um[0] + Fmb[1] * um[1] + Fmb[2] * um[2]);
  const double Xb = w[4] * Fr;
  const double phatb = Fmb[0] * n[0] + Fmb[1] * n[1] + Fmb[2] * n[2];
  const double rlnb = Frb * umn;
  const double umnb = Frb * rho_ln;
  for (int d = 0; d < 3; ++d) {
    const double Fm = phat * n[d] + um[d] * Fr;
    ab.u[d] = 0.5 * (w[4] * Fm + Fmb[d] * Fr + umnb * n[d]);
  }
  const double iblb = c1 * Xb;
  ab.k = -0.25 * Xb;
  ab.rho = 0.5 * phatb * iS + rlnb * rdx;
  ab.lrho = rlnb * rdlx;
  ab.beta = -phatb * phat * iS + iblb * bdx;
  ab.lbeta = iblb * bdlx;
}

// d(w . f(U).n)/dU for the advective flux in direction n (FP64 forward).
__host__ __device__ inline void euler_flux_vjp(const double U[5], const Prim& q, const double n[3], const double w[5],
                                               double gm1, double Ub[5]) {
  const double un = q.u[0] * n[0] + q.u[1] * n[1] + q.u[2] * n[2];
  double unb = w[0] * U[0] + w[1] * U[1] + w[2] * U[2] + w[3] * U[3] + w[4] * (U[4] + q.p);
  const double pb = w[1] * n[0] + w[2] * n[1] + w[3] * n[2] + w[4] * un;
  // direct dependence on the conserved entries
  double Ud[5] = {w[0] * un, w[1] * un, w[2] * un, w[3] * un, w[4] * un};
  const double ub[3] = {unb * n[0], unb * n[1], unb * n[2]};
  double Up[5];
  prim_vjp(q, gm1, 0.0, ub, pb, Up);
  for (int v = 0; v < 5; ++v) Ub[v] = Ud[v] + Up[v];
}

// Adjoint of the viscous flux tensor G_d[1+v] (d = 0..2, v = 0..3) with the
// weights M[d][v]: gb[12] receives d(sum M[d][v] G_d[1+v])/dg, ub[3] the
// velocity part (energy equation), and with Sutherland's law (VL 1) rpb[0],
// rpb[1] += the density and pressure parts through mu(T), lambda(T),
// T = p/(rho R).  The contracted flux Gn = sum_d n_d G_d takes M = n (x) Gnb;
// several contractions of the same flux take the sum of their M.
template <int VL = 0>
__host__ __device__ inline void viscous_tensor_vjp(const Prim& q, const double g[12], const Phys& P,
                                                   const double M[3][4], double gb[12], double ub[3],
                                                   double rpb[2] = nullptr) {
  constexpr bool suth = VL == 1;
  const double mu = suth ? visc_mu<double>(q, P) : P.mu;
  const double lam = suth ? mu * P.kappa : P.lam;
  const double divu = g[0] + g[4] + g[8];
  double tau[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) tau[a][d] = mu * (g[3 * a + d] + g[3 * d + a]);
  const double t2 = (2.0 / 3.0) * mu * divu;
  tau[0][0] -= t2; tau[1][1] -= t2; tau[2][2] -= t2;
  // taub[a][d]: weight of tau[a][d] (momentum rows, and the energy row's u . tau)
  double taub[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) taub[a][d] = M[d][a] + M[d][3] * q.u[a];
  for (int a = 0; a < 3; ++a) {
    ub[a] = 0.0;
    for (int d = 0; d < 3; ++d) ub[a] += M[d][3] * tau[d][a];
  }
  for (int c = 0; c < 12; ++c) gb[c] = 0.0;
  for (int d = 0; d < 3; ++d) gb[9 + d] = lam * M[d][3];
  double divb = 0.0;
  for (int a = 0; a < 3; ++a) divb -= (2.0 / 3.0) * mu * taub[a][a];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) {
      gb[3 * a + d] += mu * taub[a][d];
      gb[3 * d + a] += mu * taub[a][d];
    }
  gb[0] += divb; gb[4] += divb; gb[8] += divb;
  if (suth && mu != 0.0) {
    // d(weighted flux)/d mu: G is linear in mu and lambda = kappa mu
    double dmu = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int d = 0; d < 3; ++d) dmu += taub[a][d] * tau[a][d];
    dmu /= mu;
#pragma unroll
    for (int d = 0; d < 3; ++d) dmu += P.kappa * M[d][3] * g[9 + d];
    // mu = mu0 th^(3/2) (1 + Ts) / (th + Ts), th = p Rinv / (rho Tref)
    const double th = q.p * P.Rinv / (q.rho * P.Tref);
    const double thb = dmu * mu * (1.5 / th - 1.0 / (th + P.Ts));
    rpb[1] += thb * P.Rinv / (q.rho * P.Tref);
    rpb[0] -= thb * th / q.rho;
  }
}

// Adjoint of the contracted viscous flux Gn[v] = sum_d n_d G_d[1+v] with the
// weights Gnb[4] (viscous_tensor_vjp with M = n (x) Gnb).
template <int VL = 0>
__host__ __device__ inline void viscous_flux_vjp(const Prim& q, const double g[12], const Phys& P, const double n[3],
                                                 const double Gnb[4], double gb[12], double ub[3],
                                                 double rpb[2] = nullptr) {
  double M[3][4];
  for (int d = 0; d < 3; ++d)
    for (int v = 0; v < 4; ++v) M[d][v] = n[d] * Gnb[v];
  viscous_tensor_vjp<VL>(q, g, P, M, gb, ub, rpb);
}

// Adjoint of the surface flux (FP64): ULb, URb, and for Navier-Stokes gLb, gRb.
// ROE 1: Roe's dissipation; VL 1: Sutherland's law (compile-time choices,
// as in the residual).
template <int FORM, int PHYS, int ROE = 0, int VL = 0>
__host__ __device__ inline void surface_flux_vjp(const double UL[5], const double UR[5], const double* gL,
                                                 const double* gR, const double nh[3], double s, const Phys& P,
                                                 const double Phib[5], double ULb[5], double URb[5], double* gLb,
                                                 double* gRb) {
  const Prim qL = cons2prim(UL, P.gm1), qR = cons2prim(UR, P.gm1);
  const double nv[3] = {nh[0] * s, nh[1] * s, nh[2] * s};
  // central part
  if (FORM == 0 || P.twopoint == 1) {
    const double wh[5] = {0.5 * Phib[0], 0.5 * Phib[1], 0.5 * Phib[2], 0.5 * Phib[3], 0.5 * Phib[4]};
    euler_flux_vjp(UL, qL, nv, wh, P.gm1, ULb);
    euler_flux_vjp(UR, qR, nv, wh, P.gm1, URb);
  } else {
    const Aux aL = make_aux(qL), aR = make_aux(qR);
    AuxBar bL, bR;
    chandrashekar_vjp_ab(aL, aR, nv, 0.5 / P.gm1, Phib, bL, bR);
    aux_vjp(qL, aL, bL, P.gm1, ULb);
    aux_vjp(qR, aR, bR, P.gm1, URb);
  }
  // Roe's dissipation: Phi -= (s/2) D(UL, UR)
  if constexpr (ROE == 1) {
    const double Db[5] = {-0.5 * s * Phib[0], -0.5 * s * Phib[1], -0.5 * s * Phib[2], -0.5 * s * Phib[3],
                          -0.5 * s * Phib[4]};
    roe_dissipation_vjp(UL, UR, nh, P, Db, ULb, URb);
  }
  // Rusanov dissipation
  if (ROE == 0 && P.riemann == 0) {
    const double cL = sqrt(P.gamma * qL.p / qL.rho), cR = sqrt(P.gamma * qR.p / qR.rho);
    const double unL = qL.u[0] * nh[0] + qL.u[1] * nh[1] + qL.u[2] * nh[2];
    const double unR = qR.u[0] * nh[0] + qR.u[1] * nh[1] + qR.u[2] * nh[2];
    const double lL = fabs(unL) + cL, lR = fabs(unR) + cR;
    const bool left = lL >= lR;
    const double lmax = left ? lL : lR;
    const double hs = 0.5 * (lmax * s);
    double lb = 0.0;
    for (int v = 0; v < 5; ++v) {
      URb[v] -= hs * Phib[v];
      ULb[v] += hs * Phib[v];
      lb -= 0.5 * s * Phib[v] * (UR[v] - UL[v]);
    }
    const Prim& qa = left ? qL : qR;
    const double una = left ? unL : unR;
    const double ca = left ? cL : cR;
    const double sg = una >= 0.0 ? 1.0 : -1.0;
    const double ub[3] = {lb * sg * nh[0], lb * sg * nh[1], lb * sg * nh[2]};
    const double cb = lb;
    const double pb = cb * P.gamma / (2.0 * ca * qa.rho);
    const double rb = -cb * P.gamma * qa.p / (2.0 * ca * qa.rho * qa.rho);
    double Ub[5];
    prim_vjp(qa, P.gm1, rb, ub, pb, Ub);
    double* tgt = left ? ULb : URb;
    for (int v = 0; v < 5; ++v) tgt[v] += Ub[v];
  }
  if constexpr (PHYS == 1) {
    const double Gnb[4] = {-0.5 * Phib[1], -0.5 * Phib[2], -0.5 * Phib[3], -0.5 * Phib[4]};
    double ubL[3], ubR[3], rpL[2] = {0.0, 0.0}, rpR[2] = {0.0, 0.0};
    viscous_flux_vjp<VL>(qL, gL, P, nv, Gnb, gLb, ubL, rpL);
    viscous_flux_vjp<VL>(qR, gR, P, nv, Gnb, gRb, ubR, rpR);
    double Ub[5];
    prim_vjp(qL, P.gm1, rpL[0], ubL, rpL[1], Ub);
    for (int v = 0; v < 5; ++v) ULb[v] += Ub[v];
    prim_vjp(qR, P.gm1, rpR[0], ubR, rpR[1], Ub);
    for (int v = 0; v < 5; ++v) URb[v] += Ub[v];
  }
}

}  // namespace dgx

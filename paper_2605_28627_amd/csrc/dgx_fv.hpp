// dgx_fv.hpp -- FV sub-cell shock capturing for gfx950 (paper: "Governing
// Equations and Numerical Method": troubled DG elements are replaced by a
// second-order FV scheme on (N+1)^3 integral means per element, detected with
// Persson and Peraire's modal indicator; "Intra-GPU Parallelism": indicator
// and switching as element-local kernels).
//
// Scheme (one workgroup per element, one work-item per sub-cell):
//   means         mean_s = (B3 (J U))_s / V_s, B[k][i] = integral of l_i over
//                 sub-interval k; the inverse map is J U = B3^-1 (V mean)
//   reconstruction  W = (rho, u, v, w, p) per sub-cell, slope
//                 minmod(W_{k+1} - W_k, W_k - W_{k-1}) along each direction, the
//                 neighbour element's first layer as the ghost cell
//   flux          Rusanov through the sub-face vector S (not normalised)
//   residual      d mean/dt = -(1/V) sum of the outward sub-face fluxes
// Traces of an FV context carry 10 values per face node: on faces with an FV
// element on either side, the primitive means of the first two sub-cell
// layers of each side (values 0..4 and 5..9); on DG faces the DG trace.
#pragma once

#include <hip/hip_runtime.h>

#include "dgx_internal.hpp"
#include "dgx_pointwise.hpp"
#include "dgx_tile.hpp"

namespace dgx {

constexpr int kTrFV = 10;   // trace values per face node in FV contexts

__device__ __forceinline__ double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) <= fabs(b) ? a : b;
}

__device__ __forceinline__ void cons_to_prim5(const double U[5], double gm1, double W[5]) {
  const Prim q = cons2prim(U, gm1);
  W[0] = q.rho; W[1] = q.u[0]; W[2] = q.u[1]; W[3] = q.u[2]; W[4] = q.p;
}

// Rusanov flux F(WL, WR).S through the (not normalised) area vector S, from
// primitive states: the central part with S, and the dissipation
// max(|u_L.S| + c_L |S|, |u_R.S| + c_R |S|)/2 (the largest wave speed normal
// to the face times the face area) times the jump of U.
__device__ inline void rusanov_prim(const double WL[5], const double WR[5], const double S[3], const Phys& P,
                                    double F[5]) {
  const double sA = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
  double UL[5], UR[5];
  const double kL = WL[1] * WL[1] + WL[2] * WL[2] + WL[3] * WL[3];
  const double kR = WR[1] * WR[1] + WR[2] * WR[2] + WR[3] * WR[3];
  UL[0] = WL[0]; UL[1] = WL[0] * WL[1]; UL[2] = WL[0] * WL[2]; UL[3] = WL[0] * WL[3];
  UL[4] = WL[4] * P.igm1 + 0.5 * WL[0] * kL;
  UR[0] = WR[0]; UR[1] = WR[0] * WR[1]; UR[2] = WR[0] * WR[2]; UR[3] = WR[0] * WR[3];
  UR[4] = WR[4] * P.igm1 + 0.5 * WR[0] * kR;
  const double vL = WL[1] * S[0] + WL[2] * S[1] + WL[3] * S[2];
  const double vR = WR[1] * S[0] + WR[2] * S[1] + WR[3] * S[2];
  double FL[5], FR[5];
  FL[0] = UL[0] * vL; FR[0] = UR[0] * vR;
#pragma unroll
  for (int d = 0; d < 3; ++d) { FL[1 + d] = UL[1 + d] * vL + WL[4] * S[d]; FR[1 + d] = UR[1 + d] * vR + WR[4] * S[d]; }
  FL[4] = (UL[4] + WL[4]) * vL; FR[4] = (UR[4] + WR[4]) * vR;
  const double cL = sqrt(P.gamma * WL[4] / WL[0]), cR = sqrt(P.gamma * WR[4] / WR[0]);
  const double lL = fabs(vL) + cL * sA, lR = fabs(vR) + cR * sA;
  const double hs = 0.5 * (lL >= lR ? lL : lR);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - hs * (UR[v] - UL[v]);
}

// Face values of both sides of sub-face fi of an FV side (master first,
// master indexing) from their two layers: each side's first layer plus half
// its limited outward slope, the other side's first layer as ghost; and the
// master-outward sub-face vector S.
__device__ inline void fv_face_states(const double* __restrict__ Utr, const double* __restrict__ fvSb, int nS, int n2,
                                      int side, int fi, double W0f[5], double W1f[5], double S[3]) {
  double W0[2][5];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int v = 0; v < 5; ++v) W0[m][v] = Utr[tr_index(m, v, kTrFV, nS, side, n2, fi)];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double w10 = Utr[tr_index(0, 5 + v, kTrFV, nS, side, n2, fi)];
    const double w11 = Utr[tr_index(1, 5 + v, kTrFV, nS, side, n2, fi)];
    W0f[v] = W0[0][v] + 0.5 * minmod(W0[0][v] - w10, W0[1][v] - W0[0][v]);
    W1f[v] = W0[1][v] + 0.5 * minmod(W0[1][v] - w11, W0[0][v] - W0[1][v]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) S[c] = fvSb[((size_t)c * nS + side) * n2 + fi];
}

// The reconstructed face value of slot m's side alone (as in fv_face_states).
__device__ inline void fv_face_state_of(const double* __restrict__ Utr, int nS, int n2, int side, int fi, int m,
                                        double Wf[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double w0 = Utr[tr_index(m, v, kTrFV, nS, side, n2, fi)];
    const double w1 = Utr[tr_index(m, 5 + v, kTrFV, nS, side, n2, fi)];
    const double wg = Utr[tr_index(1 - m, v, kTrFV, nS, side, n2, fi)];
    Wf[v] = w0 + 0.5 * minmod(w0 - w1, wg - w0);
  }
}

// Flux through sub-face fi of an FV side, along the master normal.
__device__ inline void fv_face_flux(const double* __restrict__ Utr, const double* __restrict__ fvSb, int nS, int n2,
                                    int side, int fi, const Phys& P, double F[5]) {
  double W0f[5], W1f[5], S[3];
  fv_face_states(Utr, fvSb, nS, n2, side, fi, W0f, W1f, S);
  rusanov_prim(W0f, W1f, S, P, F);
}

// Navier-Stokes FV contexts.  The layer-0 sub-cell gradients of both sides
// of an FV face sit in gtr2[slot][12][side][fi] (component 3a+d = dq_a/dx_d,
// q = (u, v, w, T)): Green-Gauss for an FV element, the sub-cell mean of the
// lifted gradient for a DG element.  The viscous part of a sub-face flux is
// the central mean of both layer-0 sub-cells' viscous fluxes.
__device__ __forceinline__ Prim prim_of_w(const double W[5]) {
  Prim q;
  q.rho = W[0]; q.u[0] = W[1]; q.u[1] = W[2]; q.u[2] = W[3]; q.p = W[4];
  return q;
}
// F -= 1/2 (G(W0_master, g0_master) + G(W0_slave, g0_slave)) . S on sub-face fi.
__device__ inline void fv_face_visc(const double* __restrict__ Utr, const double* __restrict__ gtr2, int nS, int n2,
                                    int side, int fi, const double S[3], const Phys& P, double F[5]) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    double W[5], g[12], Gn[4];
#pragma unroll
    for (int v = 0; v < 5; ++v) W[v] = Utr[tr_index(m, v, kTrFV, nS, side, n2, fi)];
#pragma unroll
    for (int c = 0; c < 12; ++c) g[c] = gtr2[tr_index(m, c, 12, nS, side, n2, fi)];
    viscous_flux<double, 0>(prim_of_w(W), g, P, S, Gn);
#pragma unroll
    for (int v = 0; v < 4; ++v) F[1 + v] -= 0.5 * Gn[v];
  }
}

// a <- M_i a, M_j, M_k in turn (tensor product of the n1 x n1 matrix M along
// all three directions) for nvar arrays of n3 values; a and b are LDS
// buffers of nvar*n3 doubles; the result ends in b.  All work-items call it.
template <int N>
__device__ inline void tensor3(const double* M, double* a, double* b, int nvar, int t) {
  constexpr int n1 = N + 1, n2 = n1 * n1, n3 = n2 * n1;
  const bool act = t < n3;
  const int i = t % n1, j = (t / n1) % n1, k = t / n2;
  if (act)
    for (int v = 0; v < nvar; ++v) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < n1; ++l) s += M[i * n1 + l] * a[v * n3 + nidx<N>(l, j, k)];
      b[v * n3 + t] = s;
    }
  __syncthreads();
  if (act)
    for (int v = 0; v < nvar; ++v) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < n1; ++l) s += M[j * n1 + l] * b[v * n3 + nidx<N>(i, l, k)];
      a[v * n3 + t] = s;
    }
  __syncthreads();
  if (act)
    for (int v = 0; v < nvar; ++v) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < n1; ++l) s += M[k * n1 + l] * a[v * n3 + nidx<N>(i, j, l)];
      b[v * n3 + t] = s;
    }
  __syncthreads();
}

// Writes the two-layer primitive traces of the faces in face_mask (bit f =
// face f) from the primitive means sw[5][n3] in LDS.
template <int N>
__device__ inline void write_fv_traces(const Geo& G, int e, const double* sw, double* __restrict__ Utr, int face_mask,
                                       int t, int nth) {
  constexpr int n1 = N + 1, n2 = n1 * n1, n3 = n2 * n1;
  const int nS = G.nSides;
  for (int ft = t; ft < 6 * n2; ft += nth) {
    const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1, r = f / 2;
    const int info = G.efc[e * 6 + f];
    const int side = efc_side(info), slot = efc_slot(info);
    if (!((face_mask >> f) & 1)) continue;
    int p = pp, qm = qq;
    if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
    const int fi = qm * n1 + p;
    const int l0 = (f & 1) ? N : 0, l1 = (f & 1) ? N - 1 : 1;
    const int t0 = line_node<N>(r, l0, pp, qq), t1 = line_node<N>(r, l1, pp, qq);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Utr[tr_index(slot, v, kTrFV, nS, side, n2, fi)] = sw[v * n3 + t0];
      Utr[tr_index(slot, 5 + v, kTrFV, nS, side, n2, fi)] = sw[v * n3 + t1];
    }
  }
}

// ---------------------------------------------------------------------------
// Traces of an FV context: DG faces get the DG trace, FV faces the two
// primitive sub-cell layers (a DG element's from the means of its state).
// ---------------------------------------------------------------------------
// EP 1 (split form on Gauss nodes): DG faces take the entropy-projected
// trace, its ln rho, ln beta at trace_logs(Utr, nS, n2, kTrFV).
template <int N, int NODES, int EP = 0>
__global__ __launch_bounds__(Shape<N>::nth) void k_trace_fv(Geo G, Phys P, const double* __restrict__ U,
                                                            double* __restrict__ Utr) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  __shared__ double snod[5 * n3];
  __shared__ double sa[5 * n3];
  __shared__ double sb2[5 * n3];
  __shared__ double sBs[n1 * n1];
  __shared__ DevBasis sbb;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  const int nE = G.nElems, nS = G.nSides;
  const bool act = t < n3;
  load_basis(&sbb, G.basis, t, S::nth);
  for (int x = t; x < n1 * n1; x += S::nth) sBs[x] = G.basis->Bs[x];
  const int efl = G.efv[e];        // bits 0..5: FV faces, bit 6: FV element
  const int et = (efl >> 6) & 1;
  const bool anyfv = efl != 0;
  double u[5] = {0, 0, 0, 0, 0};
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = U[((size_t)v * nE + e) * n3 + t];
#pragma unroll
    for (int v = 0; v < 5; ++v) snod[v * n3 + t] = u[v];
  }
  __syncthreads();
  if (anyfv) {
    // primitive means of every sub-cell into sb2
    if (et) {
      if (act) {
        double W[5];
        cons_to_prim5(u, P.gm1, W);
#pragma unroll
        for (int v = 0; v < 5; ++v) sb2[v * n3 + t] = W[v];
      }
    } else {
      if (act) {
        const double J = 1.0 / G.sJ[(size_t)e * n3 + t];
#pragma unroll
        for (int v = 0; v < 5; ++v) sa[v * n3 + t] = J * u[v];
      }
      __syncthreads();
      tensor3<N>(sBs, sa, sb2, 5, t);
      if (act) {
        const double iv = 1.0 / G.fvV[(size_t)e * n3 + t];
        double m[5], W[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) m[v] = sb2[v * n3 + t] * iv;
        cons_to_prim5(m, P.gm1, W);
#pragma unroll
        for (int v = 0; v < 5; ++v) sb2[v * n3 + t] = W[v];
      }
    }
    __syncthreads();
    write_fv_traces<N>(G, e, sb2, Utr, et ? 63 : (efl & 63), t, S::nth);
  }
  if (et) return;
  // DG faces of a DG element: the DG trace (EP: of the entropy variables, mapped back)
  if constexpr (EP == 1) {
    if (act) {
      double w[5];
      entropy_vars(cons2prim(u, P.gm1), P.gm1, w);
#pragma unroll
      for (int v = 0; v < 5; ++v) snod[v * n3 + t] = w[v];
    }
    __syncthreads();   // (efl is uniform: every work-item gets here)
  }
  for (int ft = t; ft < S::nface; ft += S::nth) {
    const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1, r = f / 2;
    const int info = G.efc[e * 6 + f];
    const int side = efc_side(info), slot = efc_slot(info);
    if ((efl >> f) & 1) continue;
    int p = pp, q = qq;
    if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, q);
    double acc[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      acc[v] = 0.0;
      if constexpr (NODES == 1) {
        acc[v] = snod[v * n3 + line_node<N>(r, (f & 1) ? N : 0, pp, qq)];
      } else {
        const double* L = (f & 1) ? sbb.Lp : sbb.Lm;
#pragma unroll
        for (int a = 0; a < n1; ++a) acc[v] += L[a] * snod[v * n3 + line_node<N>(r, a, pp, qq)];
      }
    }
    if constexpr (EP == 1) {
      double w[5], lg[2];
#pragma unroll
      for (int v = 0; v < 5; ++v) w[v] = acc[v];
      entropy_to_cons(w, P.gm1, acc, lg);
      double* Ltr = trace_logs(Utr, nS, n2, kTrFV);
      Ltr[tr_index(slot, 0, 2, nS, side, n2, q * n1 + p)] = lg[0];
      Ltr[tr_index(slot, 1, 2, nS, side, n2, q * n1 + p)] = lg[1];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) Utr[tr_index(slot, v, kTrFV, nS, side, n2, q * n1 + p)] = acc[v];
  }
}

// ---------------------------------------------------------------------------
// Navier-Stokes, FV elements: Green-Gauss sub-cell gradients of q = (u, v, w, T),
//   g_s = (1/V_s) sum over the six sub-faces of 1/2 (q_s + q_s') S_out,
// with the neighbour element's layer-0 means across element faces (from the
// traces).  All twelve components go to gout[c][e][n3] (the FV residual
// kernel reads them), the layer-0 ones to gtr2[slot][12][side][fi].
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(Shape<N>::nth) void k_lift_fv(Geo G, Phys P, const double* __restrict__ U,
                                                           const double* __restrict__ Utr, double* __restrict__ gout,
                                                           double* __restrict__ gtr2) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  if (!G.etype[e]) return;   // DG elements belong to the lifting kernel
  const int nE = G.nElems, nS = G.nSides;
  __shared__ double sq[4 * n3];
  const bool act = t < n3;
  const int i = t % n1, j = (t / n1) % n1, k = t / n2;
  const int idx[3] = {i, j, k};
  double q[4] = {0, 0, 0, 0}, V = 1.0;
  if (act) {
    double u[5], W[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = U[((size_t)v * nE + e) * n3 + t];
    V = G.fvV[(size_t)e * n3 + t];
    cons_to_prim5(u, P.gm1, W);
    q[0] = W[1]; q[1] = W[2]; q[2] = W[3]; q[3] = W[4] / (W[0] * P.R);
#pragma unroll
    for (int c = 0; c < 4; ++c) sq[c * n3 + t] = q[c];
  }
  __syncthreads();
  if (!act) return;
  double g[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) g[c] = 0.0;
  auto add = [&](const double qf[4], const double Sv[3], double sg) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int d = 0; d < 3; ++d) g[3 * a + d] += sg * (qf[a] * Sv[d]);
  };
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int a = idx[r];
    const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
    const int rr = qq * n1 + pp;
    const int str = r == 0 ? 1 : (r == 1 ? n1 : n2);
#pragma unroll
    for (int end = 0; end < 2; ++end) {
      double qf[4], Sv[3], sg;
      const bool inner = end ? a < N : a > 0;
      if (inner) {
        // sub-face between layers kk and kk+1 along +xi_r
        const int kk = end ? a : a - 1;
        const int tn = end ? t + str : t - str;
#pragma unroll
        for (int c = 0; c < 3; ++c) Sv[c] = G.fvS[(((size_t)(3 * r + c) * nE + e) * N + kk) * n2 + rr];
        // the mean of the lower and the upper sub-cell's q
#pragma unroll
        for (int c = 0; c < 4; ++c) qf[c] = end ? 0.5 * (q[c] + sq[c * n3 + tn]) : 0.5 * (sq[c * n3 + tn] + q[c]);
        sg = end ? 1.0 : -1.0;
      } else {
        const int info = G.efc[e * 6 + 2 * r + end];
        const int side = efc_side(info), slot = efc_slot(info);
        int p = pp, qm = qq;
        if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
        const int fi = qm * n1 + p;
        double Wg[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) Wg[v] = Utr[tr_index(1 - slot, v, kTrFV, nS, side, n2, fi)];
        const double qg[4] = {Wg[1], Wg[2], Wg[3], Wg[4] / (Wg[0] * P.R)};
#pragma unroll
        for (int c = 0; c < 3; ++c) Sv[c] = G.fvSb[((size_t)c * nS + side) * n2 + fi];
#pragma unroll
        for (int c = 0; c < 4; ++c) qf[c] = 0.5 * (q[c] + qg[c]);
        sg = slot ? -1.0 : 1.0;   // outward from the master-outward vector
      }
      add(qf, Sv, sg);
    }
  }
  const double iv = 1.0 / V;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    g[c] *= iv;
    gout[((size_t)c * nE + e) * n3 + t] = g[c];
  }
  // layer-0 sub-cells: their gradient into the faces' gradient traces
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int a = idx[r];
    if (a != 0 && a != N) continue;
#pragma unroll
    for (int end = 0; end < 2; ++end) {
      if (a != (end ? N : 0)) continue;
      const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
      const int info = G.efc[e * 6 + 2 * r + end];
      const int side = efc_side(info), slot = efc_slot(info);
      int p = pp, qm = qq;
      if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
#pragma unroll
      for (int c = 0; c < 12; ++c) gtr2[tr_index(slot, c, 12, nS, side, n2, qm * n1 + p)] = g[c];
    }
  }
}

// ---------------------------------------------------------------------------
// FV elements: residual (MODE 0) or one LSERK stage and the next traces (MODE 1).
// Navier-Stokes (PHYS 1): the sub-face fluxes subtract the central mean of
// both sub-cells' viscous fluxes; the gradients come from k_lift_fv (gin,
// and gtr2 for the element faces).
// ---------------------------------------------------------------------------
template <int N, int MODE, int PHYS = 0>
__global__ __launch_bounds__(Shape<N>::nth) void k_fv(Geo G, Phys P, const double* __restrict__ U,
                                                      const double* __restrict__ Utr, const double* __restrict__ gin,
                                                      const double* __restrict__ gtr2, double* __restrict__ Ut,
                                                      double* __restrict__ Uio, double* __restrict__ dU,
                                                      double* __restrict__ Utr_next, double A, double B, double dt) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  if (!G.etype[e]) return;   // DG elements belong to the residual kernel
  const int nE = G.nElems, nS = G.nSides;
  __shared__ double sw[5 * n3];
  __shared__ double ssl[5 * n3];
  __shared__ double sfl[5 * n3];
  __shared__ double sfe[3 * 5 * n2];   // outward fluxes through the upper element faces 1, 3, 5
  __shared__ double sgr[PHYS == 1 ? 12 * n3 : 1];   // sub-cell gradients
  const bool act = t < n3;
  const int i = t % n1, j = (t / n1) % n1, k = t / n2;
  const int idx[3] = {i, j, k};
  double u[5] = {0, 0, 0, 0, 0}, W[5] = {0, 0, 0, 0, 0}, acc[5] = {0, 0, 0, 0, 0};
  double V = 1.0;
  double gme[PHYS == 1 ? 12 : 1];
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = U[((size_t)v * nE + e) * n3 + t];
    V = G.fvV[(size_t)e * n3 + t];
    if constexpr (PHYS == 1) {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        gme[c] = gin[((size_t)c * nE + e) * n3 + t];
        sgr[c * n3 + t] = gme[c];
      }
    }
  }
  // Fluxes through the three upper element faces (their loads overlap the
  // state's).  The lower element face of each line rides along with the
  // interior sub-faces below, so every direction takes one flux pass.
  for (int ft = t; ft < 3 * n2; ft += S::nth) {
    const int r = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1;
    const int info = G.efc[e * 6 + 2 * r + 1];
    const int side = efc_side(info), slot = efc_slot(info);
    int p = pp, qm = qq;
    if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
    double F[5], W0f[5], W1f[5], Sv[3];
    fv_face_states(Utr, G.fvSb, nS, n2, side, qm * n1 + p, W0f, W1f, Sv);
    rusanov_prim(W0f, W1f, Sv, P, F);
    if constexpr (PHYS == 1) fv_face_visc(Utr, gtr2, nS, n2, side, qm * n1 + p, Sv, P, F);
    const double sg = slot ? -1.0 : 1.0;   // outward
#pragma unroll
    for (int v = 0; v < 5; ++v) sfe[(r * 5 + v) * n2 + rr] = sg * F[v];
  }
  if (act) {
    cons_to_prim5(u, P.gm1, W);
#pragma unroll
    for (int v = 0; v < 5; ++v) sw[v * n3 + t] = W[v];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int a = idx[r];
    const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
    const int rr = qq * n1 + pp;
    const int str = r == 0 ? 1 : (r == 1 ? n1 : n2);
    // master index and slot of this line's two element faces
    int fi[2], side[2], slot[2];
#pragma unroll
    for (int end = 0; end < 2; ++end) {
      const int info = G.efc[e * 6 + 2 * r + end];
      side[end] = efc_side(info); slot[end] = efc_slot(info);
      int p = pp, qm = qq;
      if (slot[end]) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
      fi[end] = qm * n1 + p;
    }
    if (act) {
      double Wm[5], Wp[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        Wm[v] = a > 0 ? sw[v * n3 + t - str] : Utr[tr_index(1 - slot[0], v, kTrFV, nS, side[0], n2, fi[0])];
        Wp[v] = a < N ? sw[v * n3 + t + str] : Utr[tr_index(1 - slot[1], v, kTrFV, nS, side[1], n2, fi[1])];
        ssl[v * n3 + t] = minmod(Wp[v] - W[v], W[v] - Wm[v]);
      }
    }
    __syncthreads();
    if (act) {
      // the flux through the lower face of sub-cell a: the interior sub-face
      // (a-1 | a) along +xi_r, or for a = 0 the element face (master-outward)
      double WL[5], WR[5], Sv[3];
      if (a > 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          WL[v] = sw[v * n3 + t - str] + 0.5 * ssl[v * n3 + t - str];
          WR[v] = W[v] - 0.5 * ssl[v * n3 + t];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) Sv[c] = G.fvS[(((size_t)(3 * r + c) * nE + e) * N + a - 1) * n2 + rr];
      } else {
        fv_face_states(Utr, G.fvSb, nS, n2, side[0], fi[0], WL, WR, Sv);
      }
      double F[5];
      rusanov_prim(WL, WR, Sv, P, F);
      if constexpr (PHYS == 1) {
        if (a > 0) {
          // central mean of the two sub-cells' viscous fluxes (cell means and gradients)
          double Wl[5], gl[12], Gl[4], Gr[4];
#pragma unroll
          for (int v = 0; v < 5; ++v) Wl[v] = sw[v * n3 + t - str];
#pragma unroll
          for (int c = 0; c < 12; ++c) gl[c] = sgr[c * n3 + t - str];
          viscous_flux<double, 0>(prim_of_w(Wl), gl, P, Sv, Gl);
          viscous_flux<double, 0>(prim_of_w(W), gme, P, Sv, Gr);
#pragma unroll
          for (int v = 0; v < 4; ++v) F[1 + v] -= 0.5 * (Gl[v] + Gr[v]);
        } else {
          fv_face_visc(Utr, gtr2, nS, n2, side[0], fi[0], Sv, P, F);
        }
      }
      if (a > 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) { sfl[v * n3 + t] = F[v]; acc[v] += F[v]; }
      } else {
        const double sg = slot[0] ? -1.0 : 1.0;   // outward
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] -= sg * F[v];
      }
    }
    __syncthreads();
    if (act) {
      if (a < N) {
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] -= sfl[v * n3 + t + str];
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] -= sfe[(r * 5 + v) * n2 + rr];
      }
    }
    // (no barrier: the next direction writes sfl only after its slope barrier)
  }
  double Unew[5];
  if (act) {
    const double iv = 1.0 / V;
    if constexpr (MODE == 0) {
#pragma unroll
      for (int v = 0; v < 5; ++v) Ut[((size_t)v * nE + e) * n3 + t] = acc[v] * iv;
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const size_t gi = ((size_t)v * nE + e) * n3 + t;
        const double d = A * (A != 0.0 ? dU[gi] : 0.0) + dt * (acc[v] * iv);
        dU[gi] = d;
        Unew[v] = u[v] + B * d;
        Uio[gi] = Unew[v];
      }
      double Wn[5];
      cons_to_prim5(Unew, P.gm1, Wn);
#pragma unroll
      for (int v = 0; v < 5; ++v) sw[v * n3 + t] = Wn[v];
    }
  }
  if constexpr (MODE == 1) {
    __syncthreads();
    write_fv_traces<N>(G, e, sw, Utr_next, 63, t, S::nth);
  }
}

// ---------------------------------------------------------------------------
// Persson-Peraire indicator: log10 of the share of the modes with
// max(i,j,k) = N in the energy of rho (orthonormal Legendre basis; FV
// elements through their DG reconstruction), clamped below at -30.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(Shape<N>::nth) void k_fv_indicator(Geo G, const double* __restrict__ U,
                                                                double* __restrict__ ind) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  __shared__ double sa[n3];
  __shared__ double sb2[n3];
  __shared__ double sM[2 * n1 * n1];
  __shared__ double sred[2 * S::nth];
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  const int nE = G.nElems;
  const bool act = t < n3;
  for (int x = t; x < n1 * n1; x += S::nth) { sM[x] = G.basis->Bsi[x]; sM[n1 * n1 + x] = G.basis->Vli[x]; }
  const int et = G.etype ? G.etype[e] : 0;
  if (act) {
    const double rho = U[((size_t)0 * nE + e) * n3 + t];
    sa[t] = et ? G.fvV[(size_t)e * n3 + t] * rho : rho;
  }
  __syncthreads();
  if (et) {
    tensor3<N>(sM, sa, sb2, 1, t);
    if (act) sa[t] = sb2[t] * G.sJ[(size_t)e * n3 + t];
    __syncthreads();
  }
  tensor3<N>(sM + n1 * n1, sa, sb2, 1, t);
  const int i = t % n1, j = (t / n1) % n1, k = t / n2;
  double c2 = act ? sb2[t] * sb2[t] : 0.0;
  sred[t] = c2;
  sred[S::nth + t] = (act && (i == N || j == N || k == N)) ? c2 : 0.0;
  __syncthreads();
  // tree sum over nth entries (nth need not be a power of two)
  constexpr int p2 = S::nth <= 64 ? 64 : (S::nth <= 128 ? 128 : (S::nth <= 256 ? 256 : 512));
  for (int h = p2 / 2; h > 0; h >>= 1) {
    if (t < h && t + h < S::nth) { sred[t] += sred[t + h]; sred[S::nth + t] += sred[S::nth + t + h]; }
    __syncthreads();
  }
  if (t == 0) {
    const double r = sred[S::nth] / sred[0];
    ind[e] = log10(r > 1e-30 ? r : 1e-30);
  }
}

// ---------------------------------------------------------------------------
// Element switch: U and dU (may be null) of an element whose type changes are
// converted between nodal values and sub-cell means; its type is updated.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(Shape<N>::nth) void k_fv_switch(Geo G, double* __restrict__ U, double* __restrict__ dU,
                                                             const int* __restrict__ etype_new,
                                                             int* __restrict__ etype) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, n3 = S::n3;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  const int told = etype[e], tnew = etype_new[e];
  if (told == tnew) return;
  __shared__ double sa[5 * n3];
  __shared__ double sb2[5 * n3];
  __shared__ double sM[n1 * n1];
  const int nE = G.nElems;
  const bool act = t < n3;
  for (int x = t; x < n1 * n1; x += S::nth) sM[x] = tnew ? G.basis->Bs[x] : G.basis->Bsi[x];
  double J = 1.0, V = 1.0;
  if (act) { J = 1.0 / G.sJ[(size_t)e * n3 + t]; V = G.fvV[(size_t)e * n3 + t]; }
  for (int pass = 0; pass < 2; ++pass) {
    double* X = pass == 0 ? U : dU;
    if (!X) continue;
    if (act)
#pragma unroll
      for (int v = 0; v < 5; ++v) sa[v * n3 + t] = (tnew ? J : V) * X[((size_t)v * nE + e) * n3 + t];
    __syncthreads();
    tensor3<N>(sM, sa, sb2, 5, t);
    if (act)
#pragma unroll
      for (int v = 0; v < 5; ++v) X[((size_t)v * nE + e) * n3 + t] = sb2[v * n3 + t] / (tnew ? V : J);
    __syncthreads();
  }
  if (t == 0) etype[e] = tnew;
}

}  // namespace dgx

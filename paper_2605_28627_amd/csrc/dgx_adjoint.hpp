// dgx_adjoint.hpp -- discrete adjoint of the DGSEM residual: out = (dR/dU)^T lam.
//
// Same layout as the forward kernels (one workgroup per element, one
// work-item per node, element data in LDS).  With lt = lam / J:
//   surface:  each element writes t = -(1/w) l(+-1) lt along its normal lines
//             (k_adj_trace); the side flux's adjoint is t_master - t_slave;
//   volume:   weak form  F~^r_l gets sum_a Dhat[a][l] lt_a (transposed
//             contraction along the line); split form: node m gets
//             -sum_l J_A(m,l)^T (DS[m][l] lt_m + DS[l][m] lt_l), J_A the
//             Jacobian of F#(U_m, U_l) in its first argument (F# is symmetric);
//   lifting (Navier-Stokes): the gradient adjoint gb from the viscous terms
//             flows back through g = lift(U) (face values Qbar formed at the
//             end of the volume adjoint, then k_adj_lift_volume).
// The kinks (Rusanov's max, Roe's |.| and Harten-Hyman fix) are
// differentiated on the branch the forward takes; Sutherland's law adds the
// temperature dependence of mu and lambda.
#pragma once

#include "dgx_kernels.hpp"

namespace dgx {

// Final value a of (dR/dU)^T lam at index gi: stored in out, or (up.lamU
// set) the reverse LSERK update of the stage applied in place.  lam is
// up.lamdU then; each index is read and written by its own work-item only.
__device__ __forceinline__ double adj_store(const AdjUpd& up, double* out, size_t gi, double a) {
  if (up.lamU) {
    const double lu = up.lamU[gi] + up.dt * a;
    up.lamU[gi] = lu;
    const double ld = up.A * up.lamdU[gi] + up.Bnext * lu;
    up.lamdU[gi] = ld;
    return ld;
  }
  out[gi] = a;
  return a;
}

// Per-element surface adjoint t = -(1/w_a) l_a(+-1) (sJ lam)_a summed along
// the normal line, from sl = sJ lam [5][n3] in LDS (the element's nodes).
template <int N, int NODES>
__device__ inline void adj_surface_of(const Geo& G, const DevBasis& sb, const double* sl, int e, int t,
                                      double* __restrict__ Lbar) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  const int nS = G.nSides;
  for (int ft = t; ft < S::nface; ft += S::nth) {
    const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1, r = f / 2;
    const int info = G.efc[e * 6 + f];
    const int side = efc_side(info), slot = efc_slot(info);
    int p = pp, q = qq;
    if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, q);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double acc = 0.0;
      if constexpr (NODES == 1) {
        const int a = (f & 1) ? N : 0;
        acc = -sb.winv[a] * sl[v * n3 + line_node<N>(r, a, pp, qq)];
      } else {
        const double* L = (f & 1) ? sb.Lp : sb.Lm;
#pragma unroll
        for (int a = 0; a < n1; ++a) acc -= sb.winv[a] * L[a] * sl[v * n3 + line_node<N>(r, a, pp, qq)];
      }
      Lbar[tr_index(slot, v, 5, nS, side, n2, q * n1 + p)] = acc;
    }
  }
}

template <int N, int NODES>
__global__ __launch_bounds__(Shape<N>::nth) void k_adj_trace(Geo G, const double* __restrict__ lam,
                                                             double* __restrict__ Lbar) {
  using S = Shape<N>;
  constexpr int n3 = S::n3;
  __shared__ double sl[5 * n3];
  __shared__ DevBasis sb;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  const int nE = G.nElems;
  load_basis(&sb, G.basis, t, S::nth);
  if (t < n3) {
    const double sJ = node_metric(G, e, n3, t).sj();
#pragma unroll
    for (int v = 0; v < 5; ++v) sl[v * n3 + t] = sJ * lam[((size_t)v * nE + e) * n3 + t];
  }
  __syncthreads();
  adj_surface_of<N, NODES>(G, sb, sl, e, t, Lbar);
}

// Volume and surface adjoint of the residual.  Navier-Stokes: the gradient
// adjoint gbar (from the viscous volume and surface terms) flows back through
// the lifting g = lift(U) here as far as that is element-local: its volume
// part, out += (dq/dU)^T qbar with qbar = -sum_r Ja^r . sum_a Dhat[a][l]
// (sJ gbar)_a along the lines, and the face values of its surface part,
//   Qbar[slot][4][side][fi] = sum_a (1/w_a) l_a(+-1) sum_d (sJ gbar)_{q,d} (n s)_d,out
// along each face node's normal line, which k_adj_lift_volume takes from
// both sides of every face.
//
// Phases, so that live ranges do not stack:
//   1. each side's flux adjoint (own part) -> LDS, accumulated by the nodes;
//   2. the weak-form parts along every line (Euler weak form; the viscous
//      volume term), after which the gradients are dead; (Navier-Stokes)
//      sJ gbar -> LDS, the lifting adjoint's volume part and the faces' Qbar;
//   3. split form: per direction r the metric row -> LDS, then the pairs.
//      The weight of the pair (m, l) is w = -(DS[m][l] lt_m + DS[l][m] lt_l)
//      for both of its nodes, and F# is symmetric, so one reverse sweep of
//      F#(U_m, U_l) gives node m its first-argument and node l its
//      second-argument adjoint.  On lines inside one wavefront the lane of m
//      evaluates (m, m+d) once and hands the partner's share over a shuffle,
//      as the forward kernel does.
// Split form on Gauss nodes (the entropy-stable hybridised form): the
// element's own traces are the projected states u~_f = u(E v(U)).  Their
// adjoints collect in LDS (sub) from the surface flux (phase 1) and from the
// face coupling -(1/w_a) B_f l_f(a) (G_f(a) - S_f), G_f(a) = F#(U_a, u~_f) .
// (Ja_a + Ja_f)/2, S_f = sum_l l_f(l) G_f(l) (phase 3): with w_a the
// coupling's weight of lam_a, the coupling is sum_a (w_a - l_f(a) W) G_f(a),
// W = sum_l w_l, so each node reverses its own G_f and the u~_f parts are
// summed along the line.  Phase 4 maps them back through the projection:
// (du/dv)^T at each face node, l_f along the lines, (dv/dU)^T at each node.
// Waves per SIMD requested for 512-work-item adjoint kernels: 1 leaves the
// register file to one element per CU (the Jacobian chain stays in registers),
// 4 would cap it at 128 VGPRs for two elements per CU and spill.
#ifndef DGX_ADJ_WAVES
#define DGX_ADJ_WAVES 1
#endif
template <int N, int NODES, int FORM, int PHYS, int ROE = 0, int VL = 0>
__global__ __launch_bounds__(Shape<N>::nth, (Shape<N>::nth >= 512 ? DGX_ADJ_WAVES : 1)) void k_adj_volume(
    Geo G, Phys P, const double* __restrict__ U, const double* lam, const double* __restrict__ Utr,
    const double* __restrict__ Lbar, const double* __restrict__ gin, const double* __restrict__ gtr,
    double* __restrict__ out, double* __restrict__ Qbar, AdjUpd up) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  constexpr bool ES = FORM == 1 && NODES == 0;
  constexpr int NF = PHYS == 1 ? 17 : 5;                           // face adjoint values per face node
  constexpr int SZ_F = NF * S::nface;
  // aux (8) + one metric row (3) (+ ES: the coupling's u~_f parts of both faces, 10)
  constexpr int SZ_V = FORM == 1 ? (ES ? 21 : 11) * n3 : 0;
  constexpr int SZ_B = SZ_F > SZ_V ? SZ_F : SZ_V;
  constexpr bool kSymLines = DGX_SYMMETRIC_PAIRS && (n1 == 4 || n1 == 8) && (n3 % 64 == 0);
  // N = 7 LGL split form, Navier-Stokes: the lifting adjoint of an element
  // with constant metric terms contracts w_r = Ja^r . (gbar/J) (4 values per
  // direction and node, in sw) along the lines instead of gbar/J (12)
  constexpr bool kW = S::nth >= 512 && ROE == 0 && NODES == 1 && FORM == 1 && PHYS == 1;
  __shared__ double sl[5 * n3];   // lam / J
  __shared__ double sB[SZ_B];     // surface adjoints, then aux + metric row
  __shared__ double sw[kW ? 12 * n3 : 1];
  __shared__ double sub[ES ? 5 * S::nface : 1];   // ES: adjoints of the own projected traces
  __shared__ DevBasis sb;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  const int nE = G.nElems, nS = G.nSides;
  load_basis(&sb, G.basis, t, S::nth);
  const bool act = t < n3;
  const int i = t % n1, j = (t / n1) % n1, k = t / n2;
  const int idx[3] = {i, j, k};
  const NodeMetric nm = node_metric(G, e, n3, t);
  const double sJ = act ? nm.sj() : 0.0;
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sl[v * n3 + t] = sJ * lam[((size_t)v * nE + e) * n3 + t];
  }
  // The node's own operands of phases 2 and 3: state, metric rows, lifted
  // gradient.  In the LGL split form with one 512-work-item element per CU
  // (N = 7) the registers hold them from the start, so that their latency
  // overlaps the surface phase; elsewhere each is (re)loaded where it is
  // used, which keeps the other kernels' occupancy and spill-free budgets.
  constexpr bool kPrefetch = S::nth >= 512 && ROE == 0 && NODES == 1 && FORM == 1;
  const bool elm = kW && G.em[(size_t)9 * nE + e] > 0.0;   // constant metric terms (uniform)
  double un[5] = {0, 0, 0, 0, 0}, jn[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double gn[PHYS == 1 ? 12 : 1];
#pragma unroll
  for (int c = 0; c < (PHYS == 1 ? 12 : 1); ++c) gn[c] = 0.0;
  auto load_u = [&]() {
#pragma unroll
    for (int v = 0; v < 5; ++v) un[v] = U[((size_t)v * nE + e) * n3 + t];
  };
  auto load_row = [&](int r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) jn[3 * r + c] = nm.ja(3 * r + c);
  };
  auto load_g = [&]() {
    if constexpr (PHYS == 1) {
#pragma unroll
      for (int c = 0; c < 12; ++c) gn[c] = gin[((size_t)c * nE + e) * n3 + t];
    }
  };
  if (kPrefetch && act) {
    load_u();
    load_row(0); load_row(1); load_row(2);
    load_g();
  }
  // 1. surface: adjoint of each side's flux, own trace part into LDS.  When
  // every face node has a work-item of its own, that work-item keeps the
  // outward n s and the Qbar index of its face node for the lifting adjoint.
  constexpr bool kOneFaceNode = S::nface <= S::nth;
  double fno[3] = {0, 0, 0};
  size_t fqi = 0;
  for (int ft = t; ft < S::nface; ft += S::nth) {
    const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1;
    const int info = G.efc[e * 6 + f];
    const int side = efc_side(info), slot = efc_slot(info);
    int p = pp, qm = qq;
    if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
    const int fi = qm * n1 + p;
    double UL[5], UR[5], Phib[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      UL[v] = Utr[tr_index(0, v, 5, nS, side, n2, fi)];
      UR[v] = Utr[tr_index(1, v, 5, nS, side, n2, fi)];
      Phib[v] = Lbar[tr_index(0, v, 5, nS, side, n2, fi)] - Lbar[tr_index(1, v, 5, nS, side, n2, fi)];
    }
    double gL[12], gR[12];
    if constexpr (PHYS == 1) {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        gL[c] = gtr[tr_index(0, c, 12, nS, side, n2, fi)];
        gR[c] = gtr[tr_index(1, c, 12, nS, side, n2, fi)];
      }
    }
    const double nh[3] = {G.face[((size_t)0 * nS + side) * n2 + fi], G.face[((size_t)1 * nS + side) * n2 + fi],
                          G.face[((size_t)2 * nS + side) * n2 + fi]};
    const double s = G.face[((size_t)3 * nS + side) * n2 + fi];
    if constexpr (kOneFaceNode && PHYS == 1) {
      const double sgn = slot ? -1.0 : 1.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) fno[c] = sgn * (nh[c] * s);
      fqi = tr_index(slot, 0, 4, nS, side, n2, fi);
    }
    double ULb[5], URb[5], gLb[12], gRb[12];
    surface_flux_vjp<FORM, PHYS, ROE, VL>(UL, UR, gL, gR, nh, s, P, Phib, ULb, URb, gLb, gRb);
    // (element-wise selects keep both sides' adjoints in registers)
#pragma unroll
    for (int v = 0; v < 5; ++v) sB[(f * NF + v) * n2 + rr] = slot ? URb[v] : ULb[v];
    if constexpr (ES) {
#pragma unroll
      for (int v = 0; v < 5; ++v) sub[(f * 5 + v) * n2 + rr] = slot ? URb[v] : ULb[v];
    }
    if constexpr (PHYS == 1) {
#pragma unroll
      for (int c = 0; c < 12; ++c) sB[(f * NF + 5 + c) * n2 + rr] = slot ? gRb[c] : gLb[c];
    }
  }
  __syncthreads();
  double Ub[5] = {0, 0, 0, 0, 0};
  double gb[PHYS == 1 ? 12 : 1];
#pragma unroll
  for (int c = 0; c < (PHYS == 1 ? 12 : 1); ++c) gb[c] = 0.0;
  if (act) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int a = idx[r];
      const int rr = (r == 2 ? j : k) * n1 + (r == 0 ? j : i);
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int f = 2 * r + sd;
        double L;
        if constexpr (NODES == 1) {
          if (a != (sd ? N : 0)) continue;
          L = 1.0;
        } else {
          L = sd ? sb.Lp[a] : sb.Lm[a];
        }
        if constexpr (!ES) {   // (ES: through the projection in phase 4)
#pragma unroll
          for (int v = 0; v < 5; ++v) Ub[v] += L * sB[(f * NF + v) * n2 + rr];
        }
        if constexpr (PHYS == 1) {
#pragma unroll
          for (int c = 0; c < 12; ++c) gb[c] += L * sB[(f * NF + 5 + c) * n2 + rr];
        }
      }
    }
  }
  __syncthreads();
  // 2. weak-form parts: Lam^r = sum_a Dhat[a][l] lt_a along each line
  if (FORM == 0 || PHYS == 1) {
    if (act) {
      if (!kPrefetch) {
        load_u();
        load_g();
      }
      const double* u = un;
      const Prim q = cons2prim(u, P.gm1);
      double ub[3] = {0, 0, 0}, rpb[2] = {0.0, 0.0};
      const double* gl = gn;
      // constant viscosity: the three directions' viscous weights, summed into
      // one flux-tensor adjoint (with Sutherland's law one per direction
      // keeps fewer values live)
      double Mv[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int l = idx[r];
        const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
        double Lam[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int a = 0; a < n1; ++a) {
          const double c = sb.Dhat[a * n1 + l];
          const int ta = line_node<N>(r, a, pp, qq);
#pragma unroll
          for (int v = 0; v < 5; ++v) Lam[v] += c * sl[v * n3 + ta];
        }
        if (!kPrefetch) load_row(r);
        const double nv[3] = {jn[3 * r], jn[3 * r + 1], jn[3 * r + 2]};
        if constexpr (FORM == 0) {
          double Ue[5];
          euler_flux_vjp(u, q, nv, Lam, P.gm1, Ue);
#pragma unroll
          for (int v = 0; v < 5; ++v) Ub[v] += Ue[v];
        }
        if constexpr (PHYS == 1 && VL == 0) {
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int v = 0; v < 4; ++v) Mv[d][v] -= nv[d] * Lam[1 + v];
        } else if constexpr (PHYS == 1) {
          const double Gnb[4] = {-Lam[1], -Lam[2], -Lam[3], -Lam[4]};
          double gq[12], uq[3];
          viscous_flux_vjp<VL>(q, gl, P, nv, Gnb, gq, uq, rpb);
#pragma unroll
          for (int c = 0; c < 12; ++c) gb[c] += gq[c];
          ub[0] += uq[0]; ub[1] += uq[1]; ub[2] += uq[2];
        }
      }
      if constexpr (PHYS == 1 && VL == 0) {
        double gq[12], uq[3];
        viscous_tensor_vjp<VL>(q, gl, P, Mv, gq, uq, rpb);
#pragma unroll
        for (int c = 0; c < 12; ++c) gb[c] += gq[c];
        ub[0] += uq[0]; ub[1] += uq[1]; ub[2] += uq[2];
      }
      if constexpr (PHYS == 1) {
#pragma unroll
        for (int c = 0; c < 12; ++c) sB[c * n3 + t] = sJ * gb[c];   // (the surface adjoints in sB are consumed)
        if constexpr (kW) {
          if (elm) {
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
              for (int qa = 0; qa < 4; ++qa)
                sw[(4 * r + qa) * n3 + t] = jn[3 * r] * (sJ * gb[3 * qa]) + jn[3 * r + 1] * (sJ * gb[3 * qa + 1]) +
                                            jn[3 * r + 2] * (sJ * gb[3 * qa + 2]);
          }
        }
        double Uu[5];
        prim_vjp(q, P.gm1, rpb[0], ub, rpb[1], Uu);
#pragma unroll
        for (int v = 0; v < 5; ++v) Ub[v] += Uu[v];
      }
    }
  }
  if constexpr (PHYS == 1) {
    // the lifting adjoint's face values of this element's faces
    __syncthreads();
    const double* sg = sB;
    for (int ft = t; ft < S::nface; ft += S::nth) {
      const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1, r = f / 2;
      double no[3];
      size_t qi;
      if constexpr (kOneFaceNode) {
        no[0] = fno[0]; no[1] = fno[1]; no[2] = fno[2];
        qi = fqi;
      } else {
        const int info = G.efc[e * 6 + f];
        const int side = efc_side(info), slot = efc_slot(info);
        int p = pp, qm = qq;
        if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
        const int fi = qm * n1 + p;
        const double sgn = slot ? -1.0 : 1.0;
        const double s = G.face[((size_t)3 * nS + side) * n2 + fi];
#pragma unroll
        for (int c = 0; c < 3; ++c) no[c] = sgn * (G.face[((size_t)c * nS + side) * n2 + fi] * s);
        qi = tr_index(slot, 0, 4, nS, side, n2, fi);
      }
      double acc[4] = {0, 0, 0, 0};
#pragma unroll
      for (int a = 0; a < n1; ++a) {
        double L;
        if constexpr (NODES == 1) {
          if (a != ((f & 1) ? N : 0)) continue;
          L = sb.winv[a];
        } else {
          L = sb.winv[a] * ((f & 1) ? sb.Lp[a] : sb.Lm[a]);
        }
        const int ta = line_node<N>(r, a, pp, qq);
#pragma unroll
        for (int qa = 0; qa < 4; ++qa)
          acc[qa] += L * (sg[(3 * qa) * n3 + ta] * no[0] + sg[(3 * qa + 1) * n3 + ta] * no[1] +
                          sg[(3 * qa + 2) * n3 + ta] * no[2]);
      }
      // (values qa of one face node are nS n2 apart in the [slot][4][side][fi] layout)
#pragma unroll
      for (int qa = 0; qa < 4; ++qa) Qbar[qi + (size_t)qa * nS * n2] = acc[qa];
    }
    // the lifting adjoint's volume part: qbar = -sum_r Ja^r . (Dhat^T (sJ gbar))_r
    // (constant metric terms: -sum_r Dhat^T w_r, the transpose of the
    // lifting's factored gradient)
    if (act && kW && elm) {
      double qb[4] = {0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int l = idx[r];
        const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
#pragma unroll
        for (int a = 0; a < n1; ++a) {
          const double c = sb.Dhat[a * n1 + l];
          const int ta = line_node<N>(r, a, pp, qq);
#pragma unroll
          for (int qa = 0; qa < 4; ++qa) qb[qa] -= c * sw[(4 * r + qa) * n3 + ta];
        }
      }
      double Uq[5];
      qvars_vjp(cons2prim(un, P.gm1), P.gm1, P.Rinv, qb, Uq);
#pragma unroll
      for (int v = 0; v < 5; ++v) Ub[v] += Uq[v];
    } else if (act) {
      if (!kPrefetch) load_u();
      double qb[4] = {0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int l = idx[r];
        const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
        if (!kPrefetch) load_row(r);
        double T[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) T[c] = 0.0;
#pragma unroll
        for (int a = 0; a < n1; ++a) {
          const double c = sb.Dhat[a * n1 + l];
          const int ta = line_node<N>(r, a, pp, qq);
#pragma unroll
          for (int cc = 0; cc < 12; ++cc) T[cc] += c * sg[cc * n3 + ta];
        }
#pragma unroll
        for (int qa = 0; qa < 4; ++qa)
          qb[qa] -= jn[3 * r] * T[3 * qa] + jn[3 * r + 1] * T[3 * qa + 1] + jn[3 * r + 2] * T[3 * qa + 2];
      }
      double Uq[5];
      qvars_vjp(cons2prim(un, P.gm1), P.gm1, P.Rinv, qb, Uq);
#pragma unroll
      for (int v = 0; v < 5; ++v) Ub[v] += Uq[v];
    }
    __syncthreads();
  }
  // 3. split form: flux differencing adjoint
  if constexpr (FORM == 1) {
    double* saux = sB;
    double* sja = sB + 8 * n3;
    Aux me{};
    double lm[5] = {0, 0, 0, 0, 0};
    if (act) {
      if (!kPrefetch) load_u();
      me = make_aux(cons2prim(un, P.gm1));
      saux[0 * n3 + t] = me.rho; saux[1 * n3 + t] = me.u[0]; saux[2 * n3 + t] = me.u[1];
      saux[3 * n3 + t] = me.u[2]; saux[4 * n3 + t] = me.beta; saux[5 * n3 + t] = me.lrho;
      saux[6 * n3 + t] = me.lbeta; saux[7 * n3 + t] = me.k;
#pragma unroll
      for (int v = 0; v < 5; ++v) lm[v] = sl[v * n3 + t];
    }
    const double c1 = 0.5 / P.gm1;
    AuxBar ab{};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double jr[3] = {0, 0, 0};
      if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (!kPrefetch) jn[3 * r + c] = nm.ja(3 * r + c);
          jr[c] = jn[3 * r + c];
          sja[c * n3 + t] = jr[c];
        }
      }
      __syncthreads();
      if (act) {
        const int a = idx[r];
        const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
        auto partner = [&](int tl, Aux& ot, double nv[3]) {
          ot.rho = saux[0 * n3 + tl]; ot.u[0] = saux[1 * n3 + tl]; ot.u[1] = saux[2 * n3 + tl];
          ot.u[2] = saux[3 * n3 + tl]; ot.beta = saux[4 * n3 + tl]; ot.lrho = saux[5 * n3 + tl];
          ot.lbeta = saux[6 * n3 + tl]; ot.k = saux[7 * n3 + tl];
#pragma unroll
          for (int c = 0; c < 3; ++c) nv[c] = 0.5 * (jr[c] + sja[c * n3 + tl]);
        };
        if (P.twopoint == 0 && kSymLines && (n1 == 4 || r < 2)) {
          const int lane = t & 63;
          const int str = r == 0 ? 1 : (r == 1 ? n1 : n2);
#pragma unroll 1
          for (int d = 1; d <= n1 / 2; ++d) {
            const int b = (a + d) & (n1 - 1);
            const int tl = line_node<N>(r, b, pp, qq);
            Aux ot;
            double nv[3];
            partner(tl, ot, nv);
            const double dab = sb.DS[a * n1 + b], dba = sb.DS[b * n1 + a];
            double w[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) w[v] = -(dab * lm[v] + dba * sl[v * n3 + tl]);
            AuxBar da, db;
            chandrashekar_vjp_ab(me, ot, nv, c1, w, da, db);
            ab.rho += da.rho; ab.u[0] += da.u[0]; ab.u[1] += da.u[1]; ab.u[2] += da.u[2];
            ab.beta += da.beta; ab.lrho += da.lrho; ab.lbeta += da.lbeta; ab.k += da.k;
            if (d < n1 / 2) {
              // the lane of a - d hands over its partner share for node a
              const int src = lane + (((a - d) & (n1 - 1)) - a) * str;
              ab.rho += __shfl(db.rho, src); ab.u[0] += __shfl(db.u[0], src); ab.u[1] += __shfl(db.u[1], src);
              ab.u[2] += __shfl(db.u[2], src); ab.beta += __shfl(db.beta, src); ab.lrho += __shfl(db.lrho, src);
              ab.lbeta += __shfl(db.lbeta, src); ab.k += __shfl(db.k, src);
            }
          }
        } else {
#pragma unroll 1
          for (int l = 0; l < n1; ++l) {
            if (l == a) continue;
            const int tl = line_node<N>(r, l, pp, qq);
            Aux ot;
            double nv[3];
            partner(tl, ot, nv);
            const double dml = sb.DS[a * n1 + l], dlm = sb.DS[l * n1 + a];
            double w[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) w[v] = -(dml * lm[v] + dlm * sl[v * n3 + tl]);
            if (P.twopoint == 0) {
              AuxBar d;
              chandrashekar_vjp_a(me, ot, nv, c1, w, d);
              ab.rho += d.rho; ab.u[0] += d.u[0]; ab.u[1] += d.u[1]; ab.u[2] += d.u[2];
              ab.beta += d.beta; ab.lrho += d.lrho; ab.lbeta += d.lbeta; ab.k += d.k;
            } else {
              // central average: d/dU_m of 1/2 f(U_m).n
              if (!kPrefetch) load_u();
              const double* u = un;
              const double wh[5] = {0.5 * w[0], 0.5 * w[1], 0.5 * w[2], 0.5 * w[3], 0.5 * w[4]};
              double Ue[5];
              euler_flux_vjp(u, cons2prim(u, P.gm1), nv, wh, P.gm1, Ue);
#pragma unroll
              for (int v = 0; v < 5; ++v) Ub[v] += Ue[v];
            }
          }
        }
        if constexpr (ES) {
          // face coupling of this direction's two faces: node a reverses its
          // G_f(a) with the weight w_a - l_f(a) W; the u~_f parts go to sred
          double* sred = sB + 11 * n3;   // [2 faces][5][n3]
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const double* L = f ? sb.Lp : sb.Lm;
            const double sg = f ? -1.0 : 1.0;
            const int info = G.efc[e * 6 + 2 * r + f];
            const int side = efc_side(info), slot = efc_slot(info);
            int p = pp, qm = qq;
            if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
            double uf[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) uf[v] = Utr[tr_index(slot, v, 5, nS, side, n2, qm * n1 + p)];
            const Prim qf = cons2prim(uf, P.gm1);
            double jf[3] = {0.0, 0.0, 0.0}, W[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int l = 0; l < n1; ++l) {
              const int tl = line_node<N>(r, l, pp, qq);
              const double cw = sg * sb.winv[l] * L[l];
#pragma unroll
              for (int c = 0; c < 3; ++c) jf[c] += L[l] * sja[c * n3 + tl];
#pragma unroll
              for (int v = 0; v < 5; ++v) W[v] += cw * sl[v * n3 + tl];
            }
            const double nv[3] = {0.5 * (jr[0] + jf[0]), 0.5 * (jr[1] + jf[1]), 0.5 * (jr[2] + jf[2])};
            const double ca = sg * sb.winv[a] * L[a];
            double om[5], Uf[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) om[v] = ca * lm[v] - L[a] * W[v];
            if (P.twopoint == 0) {
              const Aux af = make_aux(qf);
              AuxBar da, dfb;
              chandrashekar_vjp_ab(me, af, nv, c1, om, da, dfb);
              ab.rho += da.rho; ab.u[0] += da.u[0]; ab.u[1] += da.u[1]; ab.u[2] += da.u[2];
              ab.beta += da.beta; ab.lrho += da.lrho; ab.lbeta += da.lbeta; ab.k += da.k;
              aux_vjp(qf, af, dfb, P.gm1, Uf);
            } else {
              if (!kPrefetch) load_u();
              const double* u = un;
              const double wh[5] = {0.5 * om[0], 0.5 * om[1], 0.5 * om[2], 0.5 * om[3], 0.5 * om[4]};
              double Ue[5];
              euler_flux_vjp(u, cons2prim(u, P.gm1), nv, wh, P.gm1, Ue);
#pragma unroll
              for (int v = 0; v < 5; ++v) Ub[v] += Ue[v];
              euler_flux_vjp(uf, qf, nv, wh, P.gm1, Uf);
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) sred[(f * 5 + v) * n3 + t] = Uf[v];
          }
        }
      }
      __syncthreads();
      if constexpr (ES) {
        // the u~_f parts of this direction's faces, summed along each line
        const double* sred = sB + 11 * n3;
        for (int ft = t; ft < 2 * n2; ft += S::nth) {
          const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1;
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < n1; ++l) acc += sred[(f * 5 + v) * n3 + line_node<N>(r, l, pp, qq)];
            sub[((2 * r + f) * 5 + v) * n2 + rr] += acc;
          }
        }
      }
    }
    if (act && P.twopoint == 0) {
      if (!kPrefetch) load_u();
      const double* u = un;
      const Prim q = cons2prim(u, P.gm1);
      double Ua[5];
      aux_vjp(q, me, ab, P.gm1, Ua);
#pragma unroll
      for (int v = 0; v < 5; ++v) Ub[v] += Ua[v];
    }
  }
  if constexpr (ES) {
    // 4. back through the projection: (du/dv)^T at each face node (v_f from
    // the projected trace), then l_f along the lines and (dv/dU)^T at each node
    __syncthreads();
    for (int ft = t; ft < S::nface; ft += S::nth) {
      const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1;
      const int info = G.efc[e * 6 + f];
      const int side = efc_side(info), slot = efc_slot(info);
      int p = pp, qm = qq;
      if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
      double uf[5], vf[5], ub[5], vb[5] = {0, 0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        uf[v] = Utr[tr_index(slot, v, 5, nS, side, n2, qm * n1 + p)];
        ub[v] = sub[(f * 5 + v) * n2 + rr];
      }
      entropy_vars(cons2prim(uf, P.gm1), P.gm1, vf);
      entropy_to_cons_vjp(vf, P.gm1, ub, vb);
#pragma unroll
      for (int v = 0; v < 5; ++v) sub[(f * 5 + v) * n2 + rr] = vb[v];
    }
    __syncthreads();
    if (act) {
      double vb[5] = {0, 0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int a = idx[r];
        const int rr = (r == 2 ? j : k) * n1 + (r == 0 ? j : i);
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          const double L = f ? sb.Lp[a] : sb.Lm[a];
#pragma unroll
          for (int v = 0; v < 5; ++v) vb[v] += L * sub[((2 * r + f) * 5 + v) * n2 + rr];
        }
      }
      if (!kPrefetch) load_u();
      const double* u = un;
      entropy_vars_vjp(u, P.gm1, vb, Ub);
    }
  }
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) adj_store(up, out, ((size_t)v * nE + e) * n3 + t, Ub[v]);
  }
}

// Lifting adjoint, face part (the volume part is in k_adj_volume):
// out += (dq/dU)^T qbar at each face node's own trace, with qbar the mean of
// both sides' Qbar.  EP 1 (split form on Gauss nodes): the face values are
// the projected traces, so their adjoints go back through the projection
// ((du/dv)^T at the face node, l_f along the line, (dv/dU)^T at the node).
// With up.lamU it is the stage's last kernel: it applies the reverse RK
// update and writes the surface adjoint of the new lamdU to up.Lnext.
template <int N, int NODES, int EP = 0>
__global__ __launch_bounds__(Shape<N>::nth) void k_adj_lift_volume(Geo G, Phys P, const double* __restrict__ U,
                                                                   const double* __restrict__ Utr,
                                                                   const double* __restrict__ Qbar,
                                                                   double* __restrict__ out, AdjUpd up) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  constexpr int SZ = 5 * S::nface > 5 * n3 ? 5 * S::nface : 5 * n3;
  __shared__ double sm[SZ];
  __shared__ DevBasis sb;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  const int nE = G.nElems, nS = G.nSides;
  load_basis(&sb, G.basis, t, S::nth);
  const bool act = t < n3;
  const int i = t % n1, j = (t / n1) % n1, k = t / n2;
  const int idx[3] = {i, j, k};
  const double sJ = act ? node_metric(G, e, n3, t).sj() : 0.0;
  double Ub[5] = {0, 0, 0, 0, 0};
  __syncthreads();
  double* sfb = sm;  // [6][5][n2]
  for (int ft = t; ft < S::nface; ft += S::nth) {
    const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1;
    const int info = G.efc[e * 6 + f];
    const int side = efc_side(info), slot = efc_slot(info);
    int p = pp, qm = qq;
    if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
    const int fi = qm * n1 + p;
    double Uo[5], qb[4];
#pragma unroll
    for (int v = 0; v < 5; ++v) Uo[v] = Utr[tr_index(slot, v, 5, nS, side, n2, fi)];
#pragma unroll
    for (int qa = 0; qa < 4; ++qa)
      qb[qa] = 0.5 * (Qbar[tr_index(0, qa, 4, nS, side, n2, fi)] + Qbar[tr_index(1, qa, 4, nS, side, n2, fi)]);
    double Ut[5];
    qvars_vjp(cons2prim(Uo, P.gm1), P.gm1, P.Rinv, qb, Ut);
    if constexpr (EP == 1) {
      double vf[5], vb[5] = {0, 0, 0, 0, 0};
      entropy_vars(cons2prim(Uo, P.gm1), P.gm1, vf);
      entropy_to_cons_vjp(vf, P.gm1, Ut, vb);
#pragma unroll
      for (int v = 0; v < 5; ++v) Ut[v] = vb[v];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sfb[(f * 5 + v) * n2 + rr] = Ut[v];
  }
  __syncthreads();
  if (act) {
    double Fb[5] = {0, 0, 0, 0, 0};   // the faces' part (EP: of the node's entropy variables)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int a = idx[r];
      const int rr = (r == 2 ? j : k) * n1 + (r == 0 ? j : i);
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int f = 2 * r + sd;
        double L;
        if constexpr (NODES == 1) {
          if (a != (sd ? N : 0)) continue;
          L = 1.0;
        } else {
          L = sd ? sb.Lp[a] : sb.Lm[a];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) Fb[v] += L * sfb[(f * 5 + v) * n2 + rr];
      }
    }
    if constexpr (EP == 1) {
      double u[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) u[v] = U[((size_t)v * nE + e) * n3 + t];
      entropy_vars_vjp(u, P.gm1, Fb, Ub);
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) Ub[v] += Fb[v];
    }
  }
  double ldn[5] = {0, 0, 0, 0, 0};   // the updated lamdU (fused update)
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const size_t gi = ((size_t)v * nE + e) * n3 + t;
      ldn[v] = adj_store(up, out, gi, out[gi] + Ub[v]);
    }
  }
  if (up.lamU && up.Lnext) {
    // the next stage's lam is the updated lamdU: its surface adjoint too
    __syncthreads();   // (sm is free once every node has read its face parts)
    if (act) {
#pragma unroll
      for (int v = 0; v < 5; ++v) sm[v * n3 + t] = sJ * ldn[v];
    }
    __syncthreads();
    adj_surface_of<N, NODES>(G, sb, sm, e, t, up.Lnext);
  }
}

}  // namespace dgx

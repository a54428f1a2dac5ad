// dgx_kernels.hpp -- HIP kernels of the DGSEM residual for gfx950.
//
// Layout: one workgroup per element, one work-item per volume node
// (i fastest), the element tile and its face data staged in LDS.  Faces are
// handled inside the element's workgroup: each side's flux is evaluated by
// both adjacent elements from the same master-ordered inputs with the same
// instructions, so both see bit-identical values and no atomics are needed.
//
// Operators (paper, "Governing Equations and Numerical Method"):
//   weak volume term   V_a += sum_l Dhat[a][l] F~^r_l,  Dhat[a][l] = (w_l/w_a) D_{l a}
//   split volume term  V_a -= sum_l DS[a][l] F#(U_a, U_l) . avg(Ja^r),  DS = M^-1 (Q - Q^T)
//   Gauss-node split   V_a -= (1/w_a) B_f l_f(a) (G_f(a) - sum_l l_f(l) G_f(l)),  f = -1, +1 ends,
//   form coupling      G_f(l) = F#(U_l, u~_f) . avg(Ja^r_l, Ja^r_f): the hybridised SBP
//                      operator with the entropy-projected face state u~_f = u(E v(U))
//   surface term       V_a -= (1/w_a) (l_a(-1) Phi^- + l_a(+1) Phi^+)   (outward Phi)
//   BR1 lifting        J g = -sum_l Dhat[a][l] (Ja^r_d q)_l + (1/w_a) l_a(+-1) {q} (n s)_d
//   residual           U_t = (V + S) / J
#pragma once

#include <hip/hip_runtime.h>

#include "dgx_internal.hpp"
#include "dgx_pointwise.hpp"
#include "dgx_tile.hpp"
#include "dgx_fv.hpp"

namespace dgx {

// The entries of the basis the residual and lifting kernels read, at their
// exact size (the LDS footprint decides how many elements share a CU).
// (FVB: also the FV sub-cell operators Bs, Bs^-1.)
template <int N, bool FVB = false>
struct VolBasis {
  static constexpr int n1 = N + 1;
  static constexpr int nf = FVB ? n1 * n1 : 1;
  double winv[n1], Lm[n1], Lp[n1], Dhat[n1 * n1], DS[n1 * n1], Bs[nf], Bsi[nf];
};
template <int N, bool FVB = false>
__device__ __forceinline__ void load_vol_basis(VolBasis<N, FVB>* dst, const DevBasis* src, int t, int nth) {
  constexpr int n1 = N + 1;
  for (int x = t; x < n1; x += nth) { dst->winv[x] = src->winv[x]; dst->Lm[x] = src->Lm[x]; dst->Lp[x] = src->Lp[x]; }
  for (int x = t; x < n1 * n1; x += nth) { dst->Dhat[x] = src->Dhat[x]; dst->DS[x] = src->DS[x]; }
  if constexpr (FVB)
    for (int x = t; x < n1 * n1; x += nth) { dst->Bs[x] = src->Bs[x]; dst->Bsi[x] = src->Bsi[x]; }
}


// ---------------------------------------------------------------------------
// Trace kernel: U at the element faces -> Utr[slot][5][side][master (p,q)].
// EP 1 (split form on Gauss nodes): the entropy-projected trace u(E v(U)),
// the entropy variables interpolated to the face and mapped back; its
// ln rho and ln beta (by-products of the map) follow the trace values in
// the same buffer (trace_logs).
// ---------------------------------------------------------------------------
template <int N, int NODES, int EP>
__global__ __launch_bounds__(Shape<N>::nth) void k_trace(Geo G, Phys P, const double* __restrict__ U,
                                                         double* __restrict__ Utr) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  const int nE = G.nElems, nS = G.nSides;
  if constexpr (NODES == 1) {
    if (t >= n3) return;
    const int i = t % n1, j = (t / n1) % n1, k = t / n2;
    const int idx[3] = {i, j, k};
    double u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = U[((size_t)v * nE + e) * n3 + t];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int a = idx[r];
      if (a != 0 && a != N) continue;
      const int f = 2 * r + (a == N ? 1 : 0);
      const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
      const int info = G.efc[e * 6 + f];
      const int side = efc_side(info), slot = efc_slot(info);
      int p = pp, q = qq;
      if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, q);
#pragma unroll
      for (int v = 0; v < 5; ++v) Utr[tr_index(slot, v, 5, nS, side, n2, q * n1 + p)] = u[v];
    }
  } else {
    __shared__ double su[5 * n3];
    __shared__ DevBasis sb;
    load_basis(&sb, G.basis, t, S::nth);
    if (t < n3) {
      double u[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) u[v] = U[((size_t)v * nE + e) * n3 + t];
      if constexpr (EP == 1) {
        double w[5];
        entropy_vars(cons2prim(u, P.gm1), P.gm1, w);
#pragma unroll
        for (int v = 0; v < 5; ++v) su[v * n3 + t] = w[v];
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) su[v * n3 + t] = u[v];
      }
    }
    __syncthreads();
    for (int ft = t; ft < S::nface; ft += S::nth) {
      const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1, r = f / 2;
      const double* L = (f & 1) ? sb.Lp : sb.Lm;
      const int info = G.efc[e * 6 + f];
      const int side = efc_side(info), slot = efc_slot(info);
      int p = pp, q = qq;
      if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, q);
      double acc[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        acc[v] = 0.0;
#pragma unroll
        for (int a = 0; a < n1; ++a) acc[v] += L[a] * su[v * n3 + line_node<N>(r, a, pp, qq)];
      }
      if constexpr (EP == 1) {
        double w[5], lg[2];
#pragma unroll
        for (int v = 0; v < 5; ++v) w[v] = acc[v];
        entropy_to_cons(w, P.gm1, acc, lg);
        double* Ltr = trace_logs(Utr, nS, n2);
        Ltr[tr_index(slot, 0, 2, nS, side, n2, q * n1 + p)] = lg[0];
        Ltr[tr_index(slot, 1, 2, nS, side, n2, q * n1 + p)] = lg[1];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) Utr[tr_index(slot, v, 5, nS, side, n2, q * n1 + p)] = acc[v];
    }
  }
}

// Viscous fluxes passed from the lifting to the residual kernel are stored in
// double (PREC 0) or, in the FP32-flux mode (PREC 1), as float in the same
// buffers (element i of the float array), like the gradients they come from.
template <int PREC>
__device__ inline void st_visc(double* p, size_t i, double v) {
  if constexpr (PREC == 1)
    reinterpret_cast<float*>(p)[i] = float(v);
  else
    p[i] = v;
}
template <int PREC>
__device__ inline double ld_visc(const double* p, size_t i) {
  if constexpr (PREC == 1)
    return double(reinterpret_cast<const float*>(p)[i]);
  else
    return p[i];
}

// ---------------------------------------------------------------------------
// BR1 lifting kernel (paper eq. dgsem_lifted), g = grad (u, v, w, T).
// EMIT 0: g -> gout[12][nE][n3] and its face traces -> gtr[slot][12][side][fi].
// EMIT 1: what the residual consumes instead of g, formed here:
//   gout[v][nE][n3] = -sum_r sum_l Dhat[a_r][l] G~^r_v(l)   (v = 0..3: the
//       viscous part of the weak-form volume term for rho u, rho v, rho w, rho e,
//       with G~^r_v = Ja^r . G_v(q, g) the contravariant viscous flux; FP64)
//   gtr[slot][4][side][fi] = G_v(q_tr, g_tr) . n s       (per side, master normal)
// with q_tr the state trace of that side.  FT is the flux arithmetic type;
// with PREC 1 the face fluxes are stored as float (st_visc).  VL is the
// viscosity law (0 constant, 1 Sutherland) of the fluxes.
//
// FV 1 (Navier-Stokes contexts with FV sub-cells; FV 2 for the split form on
// Gauss nodes, whose own face value is then the entropy-projected trace
// u(E v(U))): DG elements with an FV face only (FV 3: the DG elements
// without one, which need only the FV context's trace layout).  On a
// face whose other side is an FV element the face average takes that side's
// q as the face polynomial whose sub-face means are the q of its
// reconstructed face states (h^2 (B^-1 x B^-1), h = 2/(N+1)), and instead of
// the face-normal viscous flux the element writes the layer-0 sub-cell means
// of its gradient, B3(J g)/V, to gtr + 8 nSides n2 ([slot][12][side][fi]).
// ---------------------------------------------------------------------------
template <int N, int NODES, int EMIT, int PREC, int VL, int FV = 0>
__global__ __launch_bounds__(Shape<N>::nth) void k_lift(Geo G, Phys P, const double* __restrict__ U,
                                                        const double* __restrict__ Utr, double* __restrict__ gout,
                                                        double* __restrict__ gtr) {
  using S = Shape<N>;
  using FT = typename std::conditional<PREC == 1, float, double>::type;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  constexpr int SZ = (13 * n3 > 7 * S::nface ? 13 * n3 : 7 * S::nface);
  constexpr int SZ2 = (12 * n3 > SZ ? 12 * n3 : SZ);
  // FV 1, 2: DG elements of an FV context with an FV face (the FV-face code);
  // FV 3: those without one, in the FV context's trace layout only
  constexpr bool kCtx = FV != 0, kFvf = FV == 1 || FV == 2;
  constexpr int TNV = kCtx ? kTrFV : 5;                // trace values per face node
  __shared__ double sm[SZ2];
  __shared__ double sf[7 * S::nface];
  // FV contexts: per face node the other (FV) side's sub-face q and the own q;
  // on Gauss nodes the element's state for its own traces
  __shared__ double sfq[kFvf ? 8 * S::nface : 1];
  __shared__ double su[kFvf && NODES == 0 ? 5 * n3 : 1];
  __shared__ VolBasis<N, kFvf> sb;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  const int efl = kCtx ? G.efv[e] : 0;   // bits 0..5: FV faces, bit 6: FV element
  if (kCtx && (efl & 64)) return;        // FV elements: k_lift_fv
  if (kFvf && !(efl & 63)) return;       // (no FV face: the FV 3 variant)
  if (FV == 3 && (efl & 63)) return;
  const int nE = G.nElems, nS = G.nSides;
  load_vol_basis<N, kFvf>(&sb, G.basis, t, S::nth);
  double* sq = sm;            // [4][n3]
  double* sja = sm + 4 * n3;  // [9][n3]
  const bool act = t < n3;
  const int i = t % n1, j = (t / n1) % n1, k = t / n2;
  double sJ = 0.0;
  Prim q{};
  // Face averages {q} and outward n s of face node ft into LDS.  On LGL nodes
  // the element's own trace is its face node's state, so the own side's q is
  // read from the LDS tile (the same bits its trace would give) and only the
  // other side's trace comes from memory; on LG nodes both traces are read.
  // UO holds the other side's trace (LGL) or the master's (LG), UR the slave's (LG).
  auto face_avg = [&](int ft, int slot, const double UO[5], const double UR[5], const double nsf[4]) {
    const int f = ft / n2, rr = ft % n2;
    double qa[4], qb[4];
    {
      const Prim a = cons2prim(UO, P.gm1);
      qa[0] = a.u[0]; qa[1] = a.u[1]; qa[2] = a.u[2]; qa[3] = a.p / (a.rho * P.R);
    }
    if constexpr (NODES == 1) {
      const int pp = rr % n1, qq = rr / n1, r = f / 2;
      const int tn = line_node<N>(r, (f & 1) ? N : 0, pp, qq);
#pragma unroll
      for (int c = 0; c < 4; ++c) qb[c] = sq[c * n3 + tn];
    } else {
      const Prim b = cons2prim(UR, P.gm1);
      qb[0] = b.u[0]; qb[1] = b.u[1]; qb[2] = b.u[2]; qb[3] = b.p / (b.rho * P.R);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) sf[(f * 7 + c) * n2 + rr] = 0.5 * (qa[c] + qb[c]);
    const double sgn = slot ? -1.0 : 1.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) sf[(f * 7 + 4 + c) * n2 + rr] = sgn * (nsf[c] * nsf[3]);
  };
  auto face_load = [&](int ft, int& slot, double UO[5], double UR[5], double nsf[4]) {
    const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1;
    const int info = G.efc[e * 6 + f];
    const int side = efc_side(info);
    slot = efc_slot(info);
    int p = pp, qm = qq;
    if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
    const int fi = qm * n1 + p;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      if constexpr (NODES == 1) {
        UO[v] = Utr[tr_index(1 - slot, v, TNV, nS, side, n2, fi)];
      } else {
        UO[v] = Utr[tr_index(0, v, TNV, nS, side, n2, fi)];
        UR[v] = Utr[tr_index(1, v, TNV, nS, side, n2, fi)];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) nsf[c] = G.face[((size_t)c * nS + side) * n2 + fi];
  };
  // Every global load of this phase is issued before the first use: the
  // node's state, metrics and 1/J, and (when each face node has a work-item
  // of its own) its face node's traces and geometry.
  constexpr bool kOneFaceNode = S::nface <= S::nth;
  double u[5] = {0, 0, 0, 0, 0}, jl[9];
  double fUL[5], fUR[5], fns[4];
  int fslot = 0;
  const NodeMetric nm = node_metric(G, e, n3, t);
  const bool elm = G.em[(size_t)9 * nE + e] > 0.0;   // constant metric terms (uniform)
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = U[((size_t)v * nE + e) * n3 + t];
#pragma unroll
    for (int c = 0; c < 9; ++c) jl[c] = nm.ja(c);
    sJ = nm.sj();
  }
  if constexpr (kOneFaceNode && !kFvf) {
    if (t < S::nface) face_load(t, fslot, fUL, fUR, fns);
  }
  if (act) {
    if constexpr (FV == 1 && NODES == 0) {
#pragma unroll
      for (int v = 0; v < 5; ++v) su[v * n3 + t] = u[v];
    } else if constexpr (FV == 2) {
      double w[5];
      entropy_vars(cons2prim(u, P.gm1), P.gm1, w);
#pragma unroll
      for (int v = 0; v < 5; ++v) su[v * n3 + t] = w[v];
    }
    q = cons2prim(u, P.gm1);
    sq[0 * n3 + t] = q.u[0];
    sq[1 * n3 + t] = q.u[1];
    sq[2 * n3 + t] = q.u[2];
    sq[3 * n3 + t] = q.p / (q.rho * P.R);
#pragma unroll
    for (int c = 0; c < 9; ++c) sja[c * n3 + t] = jl[c];
  }
  // LGL: the face averages read the own q tile (FV contexts: and the own state)
  if constexpr (NODES == 1 || kFvf) __syncthreads();
  if constexpr (kFvf) {
    // FV faces: the other side's reconstructed face state at each sub-face and
    // the own trace's q into LDS; DG faces as usual
    const double h = 2.0 / n1;
    for (int ft = t; ft < S::nface; ft += S::nth) {
      const int f = ft / n2, rr = ft % n2;
      if (!((efl >> f) & 1)) {
        int slot;
        double UL[5], UR[5], nsf[4];
        face_load(ft, slot, UL, UR, nsf);
        face_avg(ft, slot, UL, UR, nsf);
        continue;
      }
      const int pp = rr % n1, qq = rr / n1, r = f / 2;
      const int info = G.efc[e * 6 + f];
      const int side = efc_side(info), slot = efc_slot(info);
      int p = pp, qm = qq;
      if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
      const int fi = qm * n1 + p;
      double Wo[5];   // the other side's reconstructed face state
      fv_face_state_of(Utr, nS, n2, side, fi, 1 - slot, Wo);
      sfq[(f * 8 + 0) * n2 + rr] = h * h * Wo[1];
      sfq[(f * 8 + 1) * n2 + rr] = h * h * Wo[2];
      sfq[(f * 8 + 2) * n2 + rr] = h * h * Wo[3];
      sfq[(f * 8 + 3) * n2 + rr] = h * h * (Wo[4] / (Wo[0] * P.R));
      double qo[4];
      if constexpr (NODES == 1) {
        const int tn = line_node<N>(r, (f & 1) ? N : 0, pp, qq);
#pragma unroll
        for (int c = 0; c < 4; ++c) qo[c] = sq[c * n3 + tn];
      } else {
        const double* L = (f & 1) ? sb.Lp : sb.Lm;
        double ut[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          ut[v] = 0.0;
#pragma unroll
          for (int a = 0; a < n1; ++a) ut[v] += L[a] * su[v * n3 + line_node<N>(r, a, pp, qq)];
        }
        if constexpr (FV == 2) {
          double w[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) w[v] = ut[v];
          entropy_to_cons(w, P.gm1, ut);
        }
        const Prim b = cons2prim(ut, P.gm1);
        qo[0] = b.u[0]; qo[1] = b.u[1]; qo[2] = b.u[2]; qo[3] = b.p / (b.rho * P.R);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) sfq[(f * 8 + 4 + c) * n2 + rr] = qo[c];
      const double sgn = slot ? -1.0 : 1.0, sA = G.face[((size_t)3 * nS + side) * n2 + fi];
#pragma unroll
      for (int c = 0; c < 3; ++c) sf[(f * 7 + 4 + c) * n2 + rr] = sgn * (G.face[((size_t)c * nS + side) * n2 + fi] * sA);
    }
    if (efl & 63) {
      __syncthreads();
      for (int ft = t; ft < S::nface; ft += S::nth) {
        const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1;
        if (!((efl >> f) & 1)) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double qf = 0.0;
          for (int q2 = 0; q2 < n1; ++q2)
#pragma unroll
            for (int p2 = 0; p2 < n1; ++p2)
              qf += sb.Bsi[pp * n1 + p2] * sb.Bsi[qq * n1 + q2] * sfq[(f * 8 + c) * n2 + q2 * n1 + p2];
          sf[(f * 7 + c) * n2 + rr] = 0.5 * (sfq[(f * 8 + 4 + c) * n2 + rr] + qf);
        }
      }
    }
  } else if constexpr (kOneFaceNode) {
    if (t < S::nface) face_avg(t, fslot, fUL, fUR, fns);
  } else {
    for (int ft = t; ft < S::nface; ft += S::nth) {
      int slot;
      double UL[5], UR[5], nsf[4];
      face_load(ft, slot, UL, UR, nsf);
      face_avg(ft, slot, UL, UR, nsf);
    }
  }
  __syncthreads();
  double acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = 0.0;
  if (act) {
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int a = idx[r];
      const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
      if (elm) {
        // constant metric terms: Ja^r times the line derivative of q, which
        // equals the contraction of Ja^r q then (4 LDS reads per line node
        // instead of 7, a third of the multiplies)
        double dq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const int tl = line_node<N>(r, l, pp, qq);
          const double c = sb.Dhat[a * n1 + l];
#pragma unroll
          for (int qa = 0; qa < 4; ++qa) dq[qa] -= c * sq[qa * n3 + tl];
        }
        const double j0 = sja[(3 * r + 0) * n3 + t], j1 = sja[(3 * r + 1) * n3 + t], j2 = sja[(3 * r + 2) * n3 + t];
#pragma unroll
        for (int qa = 0; qa < 4; ++qa) {
          acc[3 * qa + 0] += dq[qa] * j0;
          acc[3 * qa + 1] += dq[qa] * j1;
          acc[3 * qa + 2] += dq[qa] * j2;
        }
      } else {
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const int tl = line_node<N>(r, l, pp, qq);
          const double c = sb.Dhat[a * n1 + l];
          const double j0 = sja[(3 * r + 0) * n3 + tl], j1 = sja[(3 * r + 1) * n3 + tl], j2 = sja[(3 * r + 2) * n3 + tl];
#pragma unroll
          for (int qa = 0; qa < 4; ++qa) {
            const double cq = c * sq[qa * n3 + tl];
            acc[3 * qa + 0] -= cq * j0;
            acc[3 * qa + 1] -= cq * j1;
            acc[3 * qa + 2] -= cq * j2;
          }
        }
      }
      // surface terms of the two faces normal to r
#pragma unroll
      for (int side2 = 0; side2 < 2; ++side2) {
        const int f = 2 * r + side2;
        double L;
        if constexpr (NODES == 1) {
          if (a != (side2 ? N : 0)) continue;
          L = sb.winv[a];
        } else {
          L = sb.winv[a] * (side2 ? sb.Lp[a] : sb.Lm[a]);
        }
        const int rr = qq * n1 + pp;
        const double n0 = sf[(f * 7 + 4) * n2 + rr], n1v = sf[(f * 7 + 5) * n2 + rr], n2v = sf[(f * 7 + 6) * n2 + rr];
#pragma unroll
        for (int qa = 0; qa < 4; ++qa) {
          const double avg = L * sf[(f * 7 + qa) * n2 + rr];
          acc[3 * qa + 0] += avg * n0;
          acc[3 * qa + 1] += avg * n1v;
          acc[3 * qa + 2] += avg * n2v;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] *= sJ;
    if constexpr (EMIT == 0) {
#pragma unroll
      for (int c = 0; c < 12; ++c) gout[((size_t)c * nE + e) * n3 + t] = acc[c];
    }
  }
  if constexpr (EMIT == 1) {
    // Viscous part of the volume term: G~^r at every node into LDS (the
    // gradient sweep's q and Ja tiles are dead once every work-item is past
    // it), then the Dhat contraction along each node's three lines.
    double jall[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) jall[c] = act ? sja[c * n3 + t] : 0.0;
    __syncthreads();
    double* sG = sm;   // [4 r + v][n3]
    if (act) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double jr[3] = {jall[3 * r + 0], jall[3 * r + 1], jall[3 * r + 2]};
        double Gr[4];
        viscous_flux<FT, VL>(q, acc, P, jr, Gr);
#pragma unroll
        for (int v = 0; v < 4; ++v) sG[(4 * r + v) * n3 + t] = Gr[v];
      }
    }
    __syncthreads();
    if (act) {
      const int idx[3] = {i, j, k};
      double vv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int a = idx[r];
        const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const int tl = line_node<N>(r, l, pp, qq);
          const double c = sb.Dhat[a * n1 + l];
#pragma unroll
          for (int v = 0; v < 4; ++v) vv[v] -= c * sG[(4 * r + v) * n3 + tl];
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) gout[((size_t)v * nE + e) * n3 + t] = vv[v];
    }
  }
  // face-normal viscous flux of one side from its state trace qt and gradient trace gf
  auto emit_face = [&](int slot, int side, int fi, const Prim& qt, const double gf[12]) {
    const double nh[3] = {G.face[((size_t)0 * nS + side) * n2 + fi], G.face[((size_t)1 * nS + side) * n2 + fi],
                          G.face[((size_t)2 * nS + side) * n2 + fi]};
    const double s = G.face[((size_t)3 * nS + side) * n2 + fi];
    const double nv[3] = {nh[0] * s, nh[1] * s, nh[2] * s};
    double Gn[4];
    viscous_flux<FT, VL>(qt, gf, P, nv, Gn);
#pragma unroll
    for (int v = 0; v < 4; ++v) st_visc<PREC>(gtr, tr_index(slot, v, 4, nS, side, n2, fi), Gn[v]);
  };
  // gradient traces
  if constexpr (NODES == 1) {
    if (act) {
      const int idx[3] = {i, j, k};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int a = idx[r];
        if (a != 0 && a != N) continue;
        const int f = 2 * r + (a == N ? 1 : 0);
        if (kFvf && ((efl >> f) & 1)) continue;
        const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
        const int info = G.efc[e * 6 + f];
        const int side = efc_side(info), slot = efc_slot(info);
        int p = pp, qm = qq;
        if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
        if constexpr (EMIT == 0) {
#pragma unroll
          for (int c = 0; c < 12; ++c) gtr[tr_index(slot, c, 12, nS, side, n2, qm * n1 + p)] = acc[c];
        } else {
          emit_face(slot, side, qm * n1 + p, q, acc);   // LGL: the node's state is its trace
        }
      }
    }
  } else {
    __syncthreads();
    if (act)
#pragma unroll
      for (int c = 0; c < 12; ++c) sm[c * n3 + t] = acc[c];
    __syncthreads();
    for (int ft = t; ft < S::nface; ft += S::nth) {
      const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1, r = f / 2;
      if (kFvf && ((efl >> f) & 1)) continue;
      const double* L = (f & 1) ? sb.Lp : sb.Lm;
      const int info = G.efc[e * 6 + f];
      const int side = efc_side(info), slot = efc_slot(info);
      int p = pp, qm = qq;
      if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
      if constexpr (EMIT == 0) {
        for (int c = 0; c < 12; ++c) {
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < n1; ++a) s += L[a] * sm[c * n3 + line_node<N>(r, a, pp, qq)];
          gtr[tr_index(slot, c, 12, nS, side, n2, qm * n1 + p)] = s;
        }
      } else {
        double gf[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < n1; ++a) s += L[a] * sm[c * n3 + line_node<N>(r, a, pp, qq)];
          gf[c] = s;
        }
        double ut[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) ut[v] = Utr[tr_index(slot, v, TNV, nS, side, n2, qm * n1 + p)];
        emit_face(slot, side, qm * n1 + p, cons2prim(ut, P.gm1), gf);
      }
    }
  }
  if constexpr (kFvf && EMIT == 1) {
    // FV faces: layer-0 sub-cell means of the gradient, (B3 (J g))_s / V_s,
    // by a contraction along the face normal and a tensor product over the
    // face; all FV faces at once, the contractions of faces 0-2 in sf and of
    // faces 3-5 in sfq (both dead by now)
    if (efl & 63) {
      double* sjg = sm;   // [12][n3]: J g
      __syncthreads();
      if (act) {
        const double J = 1.0 / sJ;
#pragma unroll
        for (int c = 0; c < 12; ++c) sjg[c * n3 + t] = J * acc[c];
      }
      __syncthreads();
      static_assert(7 * S::nface >= 36 * n2 && 8 * S::nface >= 36 * n2, "contraction buffers");
      auto contracted = [&](int f) { return f < 3 ? sf + f * 12 * n2 : sfq + (f - 3) * 12 * n2; };
      for (int ft = t; ft < S::nface; ft += S::nth) {
        const int f = ft / n2, rr = ft % n2;
        if (!((efl >> f) & 1)) continue;
        const int r = f / 2, an = (f & 1) ? N : 0, pp = rr % n1, qq = rr / n1;
        double* T = contracted(f);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          double sacc = 0.0;
#pragma unroll
          for (int l = 0; l < n1; ++l) sacc += sb.Bs[an * n1 + l] * sjg[c * n3 + line_node<N>(r, l, pp, qq)];
          T[c * n2 + rr] = sacc;
        }
      }
      __syncthreads();
      double* gtr2 = gtr + (size_t)8 * nS * n2;
      for (int ft = t; ft < S::nface; ft += S::nth) {
        const int f = ft / n2, rr = ft % n2;
        if (!((efl >> f) & 1)) continue;
        const int r = f / 2, an = (f & 1) ? N : 0, pp = rr % n1, qq = rr / n1;
        const double* T = contracted(f);
        const int info = G.efc[e * 6 + f];
        const int side = efc_side(info), slot = efc_slot(info);
        int p = pp, qm = qq;
        if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
        const double iv = 1.0 / G.fvV[(size_t)e * n3 + line_node<N>(r, an, pp, qq)];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          double m = 0.0;
          for (int q2 = 0; q2 < n1; ++q2)
#pragma unroll
            for (int p2 = 0; p2 < n1; ++p2) m += sb.Bs[pp * n1 + p2] * sb.Bs[qq * n1 + q2] * T[c * n2 + q2 * n1 + p2];
          gtr2[tr_index(slot, c, 12, nS, side, n2, qm * n1 + p)] = m * iv;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Residual kernel: volume integral (weak or split), surface fluxes, surface
// lift, Jacobian scaling; MODE 0 writes U_t, MODE 1 applies one LSERK stage
// and writes the face traces of the new state for the next stage.
//
// Navier-Stokes: the viscous terms come from the lifting kernel (EMIT 1):
// gvn holds the viscous part of the volume term at every node (4 values),
// gvf the face-normal viscous flux of each side.
//
// Phases, so that live ranges do not stack (registers and LDS decide how
// many elements share a CU):
//   1. surface fluxes of the six faces -> LDS (before any volume state is live);
//   2. per-node two-point data -> LDS (split form);
//   3. per direction r: the metric row Ja^r -> LDS, then flux differencing
//      along r (split) or the D-hat contraction of F~^r (weak);
//   4. surface lift, the viscous volume term, 1/J, and the output or the RK stage;
//   5. face traces of the new state (RK stage).
// ---------------------------------------------------------------------------
// Symmetric evaluation of two-point pairs on lines that lie inside one
// wavefront (see k_volume); 0 evaluates every ordered pair.
#ifndef DGX_SYMMETRIC_PAIRS
#define DGX_SYMMETRIC_PAIRS 1
#endif
// Symmetric evaluation of the pairs on the zeta lines of an N = 7 element
// (they cross its eight wavefronts) with the partner shares exchanged
// through LDS; 0 evaluates every ordered pair there.
#ifndef DGX_ZETA_EXCHANGE
#define DGX_ZETA_EXCHANGE 1
#endif

// Waves per SIMD the residual kernel is compiled for (its register budget):
// 4 for elements of 512 work-items; 3 for the N = 3 Gauss split form (one
// wavefront per element), whose LDS footprint admits that many.
#ifndef DGX_ES_WAVES
#define DGX_ES_WAVES 3
#endif
// Gauss split form: the fluxes of faces 0..3 are formed in the first
// direction pass (4 n2 face nodes: all 64 lanes of an N=3 element), those of
// faces 4, 5 in the last pass, into the LDS slots of faces 0, 1, which the
// earlier passes have consumed.  Four face slots instead of six keep the
// element's LDS small enough for three waves per SIMD at N=3.
__host__ __device__ constexpr int es_face_slot(int f) { return f < 4 ? f : f - 4; }
constexpr int kEsFaceSlots = 4;
template <int N, int NODES, int FORM>
constexpr int volume_waves() {
  return Shape<N>::nth >= 512 ? 4 : ((FORM == 1 && NODES == 0 && N == 3) ? DGX_ES_WAVES : 1);
}

// FV 1 (contexts with FV sub-cells): the DG elements; for Navier-Stokes only
// those with an FV face, and FV 2 the others (which need only the FV
// context's trace layout, and run at the plain kernel's occupancy).  Faces
// with an FV element on either side take the sub-face fluxes back as the
// nodal flux polynomial (B^-1 x B^-1), and the RK epilogue writes two-layer
// primitive traces there.  Navier-Stokes: those sub-face fluxes subtract the mean of
// both layer-0 sub-cells' viscous fluxes, from the gradients at
// gvf + 8 nSides n2.
template <int N, int NODES, int FORM, int PHYS, int PREC, int MODE, int ROE, int FV = 0>
__global__ __launch_bounds__(Shape<N>::nth, (volume_waves<N, NODES, FORM>())) void k_volume(Geo G, Phys P, const double* __restrict__ U,
                                                          const double* __restrict__ Utr,
                                                          const double* __restrict__ gvn,
                                                          const double* __restrict__ gvf, double* __restrict__ Ut,
                                                          double* __restrict__ Uio, double* __restrict__ dU,
                                                          double* __restrict__ Utr_next, double A, double B,
                                                          double dt) {
  using S = Shape<N>;
  using FT = typename std::conditional<PREC == 1, float, double>::type;
  constexpr int n1 = S::n1, n2 = S::n2, n3 = S::n3;
  // split form on Gauss nodes: the entropy-stable hybridised form (face coupling terms)
  constexpr bool ES = FORM == 1 && NODES == 0;
  // lines along xi and eta (all three for n1 = 4) lie inside one wavefront
  // when n1 is a power of two and an element fills whole wavefronts
  constexpr bool kSymLines = DGX_SYMMETRIC_PAIRS && (n1 == 4 || n1 == 8) && (n3 % 64 == 0);
  // Gauss-node split form: the line sums of the face coupling go through LDS
  // (10 values per node) unless every line lies inside a wavefront
  constexpr bool kEsAllShfl = kSymLines && n1 == 4;
  // the two-point record of every node (7 values; |u|^2 is recomputed from u)
  constexpr int kAuxV = 7;
  constexpr int SZ_SPLIT = (kAuxV + 3 + (ES && !kEsAllShfl ? 10 : 0)) * n3;   // aux + Ja^r (+ face coupling)
  constexpr int SZ_WEAK = 5 * n3;                                    // F~^r
  constexpr int SZ_V = FORM == 1 ? SZ_SPLIT : SZ_WEAK;
  constexpr int SZ0 = SZ_V > 5 * n3 ? SZ_V : 5 * n3;                 // also holds the new state (Gauss traces)
  // FV: sub-face fluxes of the six faces, and two buffers for the means of the new state
  constexpr int SZ_FV = (5 * S::nface > 10 * n3 ? 5 * S::nface : 10 * n3);
  // FV 1: DG elements of an FV context (the FV-face code; Navier-Stokes:
  // those with an FV face); FV 2: Navier-Stokes DG elements without one, in
  // the FV context's trace layout only
  constexpr bool kCtx = FV != 0, kFvf = FV == 1;
  constexpr int SZ = kFvf && SZ_FV > SZ0 ? SZ_FV : SZ0;
  constexpr int TNV = kCtx ? kTrFV : 5;                              // trace values per face node
  // Surface fluxes (outward, own face-local order): all six faces at once, or
  // (Gauss split form) the two faces of each direction within its pass,
  // together with the two-point records of the own projected face states.
  // (FV contexts of the Gauss split form keep all six slots)
  constexpr int kFaces = ES && !kFvf ? kEsFaceSlots : 6;
  // Lobatto split form at N = 7: symmetric zeta pairs, partner shares through sx
  constexpr bool kZetaX = DGX_ZETA_EXCHANGE && FORM == 1 && !ES && n1 == 8 && S::nth == n3;
  __shared__ double sphi[5 * kFaces * n2];
  __shared__ double sm[SZ];
  __shared__ double sx[kZetaX ? 5 * n3 : 1];
  __shared__ double saf[ES ? 8 * kFaces * n2 : 1];
  __shared__ VolBasis<N, kFvf> sb;
  const int e = elem_of_block(blockIdx.x, G.nElems), t = threadIdx.x;
  // FV: which faces are FV (bits 0..5), and whether this element is (bit 6)
  const int efl = kCtx ? G.efv[e] : 0;
  if (kCtx && (efl & 64)) return;   // FV elements belong to the FV kernel
  if (FV == 1 && PHYS == 1 && !(efl & 63)) return;
  if (FV == 2 && (efl & 63)) return;
  const int nE = G.nElems, nS = G.nSides;
  load_vol_basis<N, kFvf>(&sb, G.basis, t, S::nth);
  const bool act = t < n3;
  const int i = t % n1, j = (t / n1) % n1, k = t / n2;
  const int idx[3] = {i, j, k};
  // Loads of the own state and of direction 0's metric row (and G~^0) are
  // issued first, so that their latency overlaps the surface fluxes; each
  // direction then prefetches the next one's while it computes.
  double u[5] = {0, 0, 0, 0, 0};
  double jn[3] = {0, 0, 0};
  // the last direction prefetches what the RK update reads instead
  double sJn = 0.0, dUn[5] = {0, 0, 0, 0, 0}, Un[5] = {0, 0, 0, 0, 0};
  // Navier-Stokes: the viscous volume term, fetched with the last direction's
  // metric row and added to the accumulator when that direction starts
  // (Gauss split form: read at the end)
  double vvn[4] = {0, 0, 0, 0};
  // (Navier-Stokes FV contexts: the node arrays, which keeps their FV-face
  // variants at N = 3 and 5 within four waves per SIMD)
  constexpr bool kElemM = FV == 0 || PHYS == 0;
  const NodeMetric nm = node_metric<kElemM>(G, e, n3, t);
  auto fetch_end = [&]() {
    if constexpr (kElemM)
      sJn = nm.sj();
    else
      sJn = G.sJ[(size_t)e * n3 + t];
    if constexpr (MODE == 1) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const size_t gi = ((size_t)v * nE + e) * n3 + t;
        dUn[v] = A != 0.0 ? dU[gi] : 0.0;   // the first LSERK stage has A = 0: no read
        Un[v] = U[gi];
      }
    }
  };
  auto fetch_dir = [&](int r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (kElemM)
        jn[c] = nm.ja(3 * r + c);
      else
        jn[c] = G.Ja[((size_t)(3 * r + c) * nE + e) * n3 + t];
    }
    if constexpr (PHYS == 1 && !ES) {
      if (r == 2) {
#pragma unroll
        for (int v = 0; v < 4; ++v) vvn[v] = gvn[((size_t)v * nE + e) * n3 + t];
      }
    }
  };
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = U[((size_t)v * nE + e) * n3 + t];
    fetch_dir(0);
  }
  // surface flux of face f at its node rr into LDS slot fs (and, ES, the own record)
  auto face_node = [&](int f, int rr, int fs) {
    const int pp = rr % n1, qq = rr / n1;
    const int info = G.efc[e * 6 + f];
    const int side = efc_side(info), slot = efc_slot(info);
    int p = pp, qm = qq;
    if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
    const int fi = qm * n1 + p;
    if constexpr (kFvf) {
      if ((efl >> f) & 1) {
        // FV face: the sub-face flux, outward, into the staging area (taken back below);
        // Navier-Stokes: less the mean of both layer-0 sub-cells' viscous fluxes
        double F[5], W0f[5], W1f[5], Sv[3];
        fv_face_states(Utr, G.fvSb, nS, n2, side, fi, W0f, W1f, Sv);
        rusanov_prim(W0f, W1f, Sv, P, F);
        if constexpr (PHYS == 1) fv_face_visc(Utr, gvf + (size_t)8 * nS * n2, nS, n2, side, fi, Sv, P, F);
        const double so = slot ? -1.0 : 1.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) sm[(f * 5 + v) * n2 + rr] = so * F[v];
        return;
      }
    }
    double UL[5], UR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      UL[v] = Utr[tr_index(0, v, TNV, nS, side, n2, fi)];
      UR[v] = Utr[tr_index(1, v, TNV, nS, side, n2, fi)];
    }
    const double nh[3] = {G.face[((size_t)0 * nS + side) * n2 + fi], G.face[((size_t)1 * nS + side) * n2 + fi],
                          G.face[((size_t)2 * nS + side) * n2 + fi]};
    const double s = G.face[((size_t)3 * nS + side) * n2 + fi];
    double Phi[5];
    Aux own;
    if constexpr (ES) {
      // the projected traces carry their ln rho, ln beta
      const double* Ltr = trace_logs(Utr, nS, n2, TNV);
      const double lg[4] = {Ltr[tr_index(0, 0, 2, nS, side, n2, fi)], Ltr[tr_index(0, 1, 2, nS, side, n2, fi)],
                            Ltr[tr_index(1, 0, 2, nS, side, n2, fi)], Ltr[tr_index(1, 1, 2, nS, side, n2, fi)]};
      surface_flux_adv<FT, FORM, ROE>(UL, UR, nh, s, P, Phi, &own, slot, lg);
    } else {
      surface_flux_adv<FT, FORM, ROE>(UL, UR, nh, s, P, Phi);
    }
    if constexpr (ES) {
      double* d = saf + fs * 8 * n2 + rr;
      d[0] = own.rho; d[n2] = own.u[0]; d[2 * n2] = own.u[1]; d[3 * n2] = own.u[2];
      d[4 * n2] = own.beta; d[5 * n2] = own.lrho; d[6 * n2] = own.lbeta; d[7 * n2] = own.k;
    }
    if constexpr (PHYS == 1) {
      // face-normal viscous fluxes of the two sides, formed by the lifting
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int v = 0; v < 4; ++v) Phi[1 + v] -= 0.5 * ld_visc<PREC>(gvf, tr_index(sd, v, 4, nS, side, n2, fi));
    }
    const double sgn = slot ? -1.0 : 1.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) sphi[(fs * 5 + v) * n2 + rr] = sgn * Phi[v];
  };
  // 1. surface fluxes of the six faces (other forms)
  if constexpr (!ES) {
    for (int ft = t; ft < S::nface; ft += S::nth) face_node(ft / n2, ft % n2, ft / n2);
  }
  if constexpr (ES && kFvf) {
    if (efl & 63) {
      // FV faces of the Gauss split form: the traces there hold sub-cell
      // means, so the element forms the two-point records of its own
      // entropy-projected face states u(E v(U)) for the face coupling here
      // (the same arithmetic as its traces on DG faces), then the sub-face fluxes.
      if (act) {
        double w[5];
        entropy_vars(cons2prim(u, P.gm1), P.gm1, w);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm[v * n3 + t] = w[v];
      }
      __syncthreads();
      for (int ft = t; ft < S::nface; ft += S::nth) {
        const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1, r = f / 2;
        if (!((efl >> f) & 1)) continue;
        const double* L = (f & 1) ? sb.Lp : sb.Lm;
        double w[5], uf[5], lg[2];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          w[v] = 0.0;
#pragma unroll
          for (int a = 0; a < n1; ++a) w[v] += L[a] * sm[v * n3 + line_node<N>(r, a, pp, qq)];
        }
        entropy_to_cons(w, P.gm1, uf, lg);
        const Prim qf = cons2prim(uf, P.gm1);
        const Aux own = P.twopoint == 0 ? make_aux_logs(qf, lg[0], lg[1]) : make_aux(qf);
        double* d = saf + f * 8 * n2 + rr;
        d[0] = own.rho; d[n2] = own.u[0]; d[2 * n2] = own.u[1]; d[3 * n2] = own.u[2];
        d[4 * n2] = own.beta; d[5 * n2] = own.lrho; d[6 * n2] = own.lbeta; d[7 * n2] = own.k;
      }
      __syncthreads();
      for (int ft = t; ft < S::nface; ft += S::nth)
        if ((efl >> (ft / n2)) & 1) face_node(ft / n2, ft % n2, ft / n2);
    }
  }
  if constexpr (kFvf) {
    // FV faces: nodal flux polynomial with the sub-face integrals, Phi = (B^-1 x B^-1) F
    __syncthreads();
    for (int ft = t; ft < S::nface; ft += S::nth) {
      const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1;
      if (!((efl >> f) & 1)) continue;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double sacc = 0.0;
        for (int q2 = 0; q2 < n1; ++q2)
#pragma unroll
          for (int p2 = 0; p2 < n1; ++p2)
            sacc += sb.Bsi[pp * n1 + p2] * sb.Bsi[qq * n1 + q2] * sm[(f * 5 + v) * n2 + q2 * n1 + p2];
        sphi[(f * 5 + v) * n2 + rr] = sacc;
      }
    }
    __syncthreads();
  }
  // 2. own state
  double acc[5] = {0, 0, 0, 0, 0};
  Prim q{};
  if (act) q = cons2prim(u, P.gm1);
  Aux me{};
  if constexpr (FORM == 1) {
    if (act) {
      me = make_aux(q);
      sm[0 * n3 + t] = me.rho; sm[1 * n3 + t] = me.u[0]; sm[2 * n3 + t] = me.u[1]; sm[3 * n3 + t] = me.u[2];
      sm[4 * n3 + t] = me.beta; sm[5 * n3 + t] = me.lrho; sm[6 * n3 + t] = me.lbeta;
    }
  }
  // 3. volume integral, one reference direction at a time (unrolled: the
  // line strides and the symmetric-pair choice are then constants)
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double jr[3] = {jn[0], jn[1], jn[2]};
    if constexpr (PHYS == 1 && !ES) {
      if (r == 2 && act) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[1 + v] += vvn[v];
      }
    }
    if constexpr (FORM == 1) {
      double* sja = sm + kAuxV * n3;
      if constexpr (ES) {
        // the faces whose flux is formed in this pass: 0..3 in the first, 4, 5 in the last
        constexpr int fa[3] = {0, 6, 4}, fb[3] = {4, 6, 6};
        for (int ft = fa[r] * n2 + t; ft < fb[r] * n2; ft += S::nth) {
          if (kFvf && ((efl >> (ft / n2)) & 1)) continue;   // formed in step 1
          face_node(ft / n2, ft % n2, kFvf ? ft / n2 : es_face_slot(ft / n2));
        }
      }
      if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) sja[c * n3 + t] = jr[c];
      }
      __syncthreads();
      if (act) {
        if (r < 2) fetch_dir(r + 1);
        else fetch_end();
      }
      double Gf[2][5];   // face coupling of this node (ES)
      if (act) {
        const int a = idx[r];
        const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
        const double c1 = 0.5 / P.gm1;
        // two-point flux F#(U_a, ot) . nv
        auto two_point = [&](const Aux& ot, const double nv[3], double F[5]) {
          if (P.twopoint == 0) {
            chandrashekar<FT>(me, ot, nv, c1, F, P.p0, P.ib0);
          } else {
            // central average of the two physical fluxes (states rebuilt from the staged data)
            double Fa[5], Fb[5];
            aux_flux<FT>(me, P.gm1, nv, Fa);
            aux_flux<FT>(ot, P.gm1, nv, Fb);
#pragma unroll
            for (int v = 0; v < 5; ++v) F[v] = 0.5 * (Fa[v] + Fb[v]);
          }
        };
        // two-point flux F#(U_a, U_l) . avg(Ja^r) with the partner node tl
        auto pair_flux = [&](int tl, double F[5]) {
          Aux ot;
          ot.rho = sm[0 * n3 + tl]; ot.u[0] = sm[1 * n3 + tl]; ot.u[1] = sm[2 * n3 + tl];
          ot.u[2] = sm[3 * n3 + tl]; ot.beta = sm[4 * n3 + tl]; ot.lrho = sm[5 * n3 + tl];
          ot.lbeta = sm[6 * n3 + tl];
          ot.k = ot.u[0] * ot.u[0] + ot.u[1] * ot.u[1] + ot.u[2] * ot.u[2];
          const double nv[3] = {0.5 * (jr[0] + sja[0 * n3 + tl]), 0.5 * (jr[1] + sja[1 * n3 + tl]),
                                0.5 * (jr[2] + sja[2 * n3 + tl])};
          two_point(ot, nv, F);
        };
        if (kSymLines && (n1 == 4 || r < 2)) {
          // The line lies inside this wavefront, its nodes kStride apart in
          // lanes.  F# is symmetric in its two states, so the pair (a, a+d) is
          // evaluated once, by the lane of a: it keeps -DS[a][a+d] F and hands
          // -DS[a+d][a] F to the lane of a+d, receiving the share of the pair
          // (a-d, a) in turn.  The pair at distance n1/2 is met from both ends
          // and each lane keeps its own share.
          const int lane = t & 63;
          const int str = r == 0 ? 1 : (r == 1 ? n1 : n2);
#pragma unroll 1
          for (int d = 1; d <= n1 / 2; ++d) {
            const int b = (a + d) & (n1 - 1);
            double F[5];
            pair_flux(line_node<N>(r, b, pp, qq), F);
            const double dab = sb.DS[a * n1 + b];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[v] -= dab * F[v];
            if (d < n1 / 2) {
              const double dba = sb.DS[b * n1 + a];
              const int src = lane + (((a - d) & (n1 - 1)) - a) * str;
#pragma unroll
              for (int v = 0; v < 5; ++v) acc[v] += __shfl(-dba * F[v], src);
            }
          }
        } else if (kZetaX && r == 2) {
          // The zeta line crosses the element's waves: the pair (a, a+d) is
          // evaluated once, by the node of a, which hands -DS[a+d][a] F to
          // the node of a+d through sx (every node of the block takes part:
          // the element fills it).  Distance n1/2 is met from both ends.
#pragma unroll 1
          for (int d = 1; d <= n1 / 2; ++d) {
            const int b = (a + d) & (n1 - 1);
            const int tb = line_node<N>(r, b, pp, qq);
            double F[5];
            pair_flux(tb, F);
            const double dab = sb.DS[a * n1 + b];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[v] -= dab * F[v];
            if (d < n1 / 2) {
              const double dba = sb.DS[b * n1 + a];
#pragma unroll
              for (int v = 0; v < 5; ++v) sx[v * n3 + tb] = -dba * F[v];
              __syncthreads();
#pragma unroll
              for (int v = 0; v < 5; ++v) acc[v] += sx[v * n3 + t];
              __syncthreads();
            }
          }
        } else {
          for (int l = 0; l < n1; ++l) {
            const int tl = line_node<N>(r, l, pp, qq);
            if (l == a) continue;
            double F[5];
            pair_flux(tl, F);
            const double ds = sb.DS[a * n1 + l];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[v] -= ds * F[v];
          }
        }
        if constexpr (ES) {
          // Face coupling of the hybridised operator: G_f = F#(U_a, u~_f) . (Ja^r_a + Ja^r_f)/2
          // with u~_f the projected face state and Ja^r_f the metric row
          // interpolated to the end f of this line; l_f(a) G_f is staged for
          // the line sums S_f = sum_l l_f(l) G_f(l).
          // The surface term of this direction's two faces is applied here too.
          double* shy = sm + (kAuxV + 3) * n3;
          const int rr = qq * n1 + pp;
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const double* L = f ? sb.Lp : sb.Lm;
            const double cs = sb.winv[a] * L[a];
            const int fsl = kFvf ? 2 * r + f : es_face_slot(2 * r + f);
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[v] -= cs * sphi[(fsl * 5 + v) * n2 + rr];
            double jf[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int l = 0; l < n1; ++l) {
              const int tl = line_node<N>(r, l, pp, qq);
#pragma unroll
              for (int c = 0; c < 3; ++c) jf[c] += L[l] * sja[c * n3 + tl];
            }
            const double* d = saf + fsl * 8 * n2 + rr;
            Aux of;
            of.rho = d[0]; of.u[0] = d[n2]; of.u[1] = d[2 * n2]; of.u[2] = d[3 * n2];
            of.beta = d[4 * n2]; of.lrho = d[5 * n2]; of.lbeta = d[6 * n2]; of.k = d[7 * n2];
            const double nv[3] = {0.5 * (jr[0] + jf[0]), 0.5 * (jr[1] + jf[1]), 0.5 * (jr[2] + jf[2])};
            two_point(of, nv, Gf[f]);
            if (kSymLines && (n1 == 4 || r < 2)) {
              // line sum by a butterfly over the line's lanes (bits of a in the lane id)
              const int str = r == 0 ? 1 : (r == 1 ? n1 : n2);
              const double cf = (f ? 1.0 : -1.0) * sb.winv[a] * L[a];
#pragma unroll
              for (int v = 0; v < 5; ++v) {
                double x = L[a] * Gf[f][v];
#pragma unroll
                for (int m = 1; m < n1; m <<= 1) x += __shfl_xor(x, m * str);
                acc[v] -= cf * (Gf[f][v] - x);
              }
            } else {
#pragma unroll
              for (int v = 0; v < 5; ++v) shy[(f * 5 + v) * n3 + t] = L[a] * Gf[f][v];
            }
          }
        }
      }
      if (ES && !(kSymLines && (n1 == 4 || r < 2))) {
        // dU_a -= (1/w_a) B_f l_f(a) (G_f(a) - S_f),  B_f = -1 at xi = -1, +1 at xi = +1
        __syncthreads();
        if (act) {
          const double* shy = sm + (kAuxV + 3) * n3;
          const int a = idx[r];
          const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const double cf = (f ? 1.0 : -1.0) * sb.winv[a] * (f ? sb.Lp[a] : sb.Lm[a]);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
              double Sf = 0.0;
#pragma unroll
              for (int l = 0; l < n1; ++l) Sf += shy[(f * 5 + v) * n3 + line_node<N>(r, l, pp, qq)];
              acc[v] -= cf * (Gf[f][v] - Sf);
            }
          }
        }
      }
      __syncthreads();
    } else {
      // weak form: F~^r = Ja^r . f at every node, then the Dhat contraction
      // (the viscous part comes contracted from the lifting kernel)
      if (act) {
        double F[5];
        euler_flux<FT>(u, q, jr, F, P.p0, P.h0);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm[v * n3 + t] = F[v];
      }
      __syncthreads();
      if (act) {
        if (r < 2) fetch_dir(r + 1);
        else fetch_end();
      }
      if (act) {
        const int a = idx[r];
        const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const int tl = line_node<N>(r, l, pp, qq);
          const double c = sb.Dhat[a * n1 + l];
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v] += c * sm[v * n3 + tl];
        }
      }
      __syncthreads();
    }
  }
  // 4. surface lift (other forms), Jacobian, output
  double Unew[5];
  if (act) {
#pragma unroll
    for (int r = 0; r < (ES ? 0 : 3); ++r) {
      const int a = idx[r];
      const int rr = (r == 2 ? j : k) * n1 + (r == 0 ? j : i);
      if constexpr (NODES == 1) {
        if (a == 0) {
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v] -= sb.winv[0] * sphi[((2 * r) * 5 + v) * n2 + rr];
        }
        if (a == N) {
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v] -= sb.winv[N] * sphi[((2 * r + 1) * 5 + v) * n2 + rr];
        }
      } else {
        const double cm = sb.winv[a] * sb.Lm[a], cp = sb.winv[a] * sb.Lp[a];
#pragma unroll
        for (int v = 0; v < 5; ++v)
          acc[v] -= cm * sphi[((2 * r) * 5 + v) * n2 + rr] + cp * sphi[((2 * r + 1) * 5 + v) * n2 + rr];
      }
    }
    if constexpr (PHYS == 1 && ES) {
      // (Gauss split form: read here, where fewer values are live)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[1 + v] += gvn[((size_t)v * nE + e) * n3 + t];
    }
    const double sJ = sJn;
    if constexpr (MODE == 0) {
#pragma unroll
      for (int v = 0; v < 5; ++v) Ut[((size_t)v * nE + e) * n3 + t] = acc[v] * sJ;
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const size_t gi = ((size_t)v * nE + e) * n3 + t;
        const double d = A * dUn[v] + dt * (acc[v] * sJ);
        dU[gi] = d;
        Unew[v] = Un[v] + B * d;
        Uio[gi] = Unew[v];
      }
    }
  }
  // 5. traces of the new state for the next stage
  if constexpr (MODE == 1) {
    if constexpr (NODES == 1) {
      if (act) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const int a = idx[r];
          if (a != 0 && a != N) continue;
          const int f = 2 * r + (a == N ? 1 : 0);
          const int pp = r == 0 ? j : i, qq = r == 2 ? j : k;
          const int info = G.efc[e * 6 + f];
          const int side = efc_side(info), slot = efc_slot(info);
          if (kFvf && ((efl >> f) & 1)) continue;
          int p = pp, qm = qq;
          if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
#pragma unroll
          for (int v = 0; v < 5; ++v) Utr_next[tr_index(slot, v, TNV, nS, side, n2, qm * n1 + p)] = Unew[v];
        }
      }
    } else {
      // (entropy-projected traces in the split form)
      if (act) {
        double w[5];
        if constexpr (ES) {
          entropy_vars(cons2prim(Unew, P.gm1), P.gm1, w);
        } else {
#pragma unroll
          for (int v = 0; v < 5; ++v) w[v] = Unew[v];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) sm[v * n3 + t] = w[v];
      }
      __syncthreads();
      for (int ft = t; ft < S::nface; ft += S::nth) {
        const int f = ft / n2, rr = ft % n2, pp = rr % n1, qq = rr / n1, r = f / 2;
        const double* L = (f & 1) ? sb.Lp : sb.Lm;
        const int info = G.efc[e * 6 + f];
        const int side = efc_side(info), slot = efc_slot(info);
        if (kFvf && ((efl >> f) & 1)) continue;
        int p = pp, qm = qq;
        if (slot) orient_to_master(efc_orient(info), N, pp, qq, p, qm);
        double s[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          s[v] = 0.0;
#pragma unroll
          for (int a = 0; a < n1; ++a) s[v] += L[a] * sm[v * n3 + line_node<N>(r, a, pp, qq)];
        }
        if constexpr (ES) {
          double w[5], lg[2];
#pragma unroll
          for (int v = 0; v < 5; ++v) w[v] = s[v];
          entropy_to_cons(w, P.gm1, s, lg);
          double* Ltr = trace_logs(Utr_next, nS, n2, TNV);
          Ltr[tr_index(slot, 0, 2, nS, side, n2, qm * n1 + p)] = lg[0];
          Ltr[tr_index(slot, 1, 2, nS, side, n2, qm * n1 + p)] = lg[1];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) Utr_next[tr_index(slot, v, TNV, nS, side, n2, qm * n1 + p)] = s[v];
      }
    }
    if constexpr (kFvf) {
      // FV faces of this DG element: primitive means of its first two sub-cell layers
      const bool anyfv = (efl & 63) != 0;
      if (anyfv) {
        __syncthreads();
        double* sa = sm;
        double* sc = sm + 5 * n3;
        if (act) {
          const double J = 1.0 / sJn;
#pragma unroll
          for (int v = 0; v < 5; ++v) sa[v * n3 + t] = J * Unew[v];
        }
        __syncthreads();
        tensor3<N>(sb.Bs, sa, sc, 5, t);
        if (act) {
          const double iv = 1.0 / G.fvV[(size_t)e * n3 + t];
          double m[5], W[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) m[v] = sc[v * n3 + t] * iv;
          cons_to_prim5(m, P.gm1, W);
#pragma unroll
          for (int v = 0; v < 5; ++v) sc[v * n3 + t] = W[v];
        }
        __syncthreads();
        write_fv_traces<N>(G, e, sc, Utr_next, efl & 63, t, S::nth);
      }
    }
  }
}

}  // namespace dgx

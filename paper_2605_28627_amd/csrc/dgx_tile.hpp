// dgx_tile.hpp -- element-tile index helpers shared by the residual and FV
// kernels: work-items per element, node and line indexing, the basis copy,
// and the face-trace layout.
#pragma once

#include <hip/hip_runtime.h>

#include "dgx_internal.hpp"

namespace dgx {

template <int N>
struct Shape {
  static constexpr int n1 = N + 1;
  static constexpr int n2 = n1 * n1;
  static constexpr int n3 = n2 * n1;
  static constexpr int nth = ((n3 + 63) / 64) * 64;   // work-items per element (whole wavefronts)
  static constexpr int nface = 6 * n2;                 // face nodes of one element
};

template <int N>
__device__ __forceinline__ int nidx(int i, int j, int k) { return (k * (N + 1) + j) * (N + 1) + i; }

// Volume node at position a along reference direction r, tangential face indices (pp, qq).
template <int N>
__device__ __forceinline__ int line_node(int r, int a, int pp, int qq) {
  return r == 0 ? nidx<N>(a, pp, qq) : (r == 1 ? nidx<N>(pp, a, qq) : nidx<N>(pp, qq, a));
}

// Copy the basis into LDS (cooperatively).
__device__ __forceinline__ void load_basis(DevBasis* dst, const DevBasis* src, int t, int nth) {
  const double* s = reinterpret_cast<const double*>(src);
  double* d = reinterpret_cast<double*>(dst);
  constexpr int nd = sizeof(DevBasis) / sizeof(double);
  for (int x = t; x < nd; x += nth) d[x] = s[x];
}

// Where node t of element e finds its metric terms: component c (Ja^r_n at
// c = 3r+n, 1/J at c = 9) at base[off + c st].  Both stores are [10][...]:
// the node arrays (Ja, then sJ) and, for every element whose terms are the
// same at all of its nodes (affine), the per-element copy G.em, whose 1/J is
// positive exactly for those elements.  Such an element's nodes all read the
// copy and the node arrays are not touched (same values).
// Selects only, no branches; base and st are uniform over the workgroup.
struct NodeMetric {
  const double* base;
  size_t off, st;
  __device__ __forceinline__ double ja(int c) const { return base[off + c * st]; }
  __device__ __forceinline__ double sj() const { return base[off + 9 * st]; }
};
// ELEM = false: always the node arrays (kernels whose register budget has no
// room for the selects).
template <bool ELEM = true>
__device__ __forceinline__ NodeMetric node_metric(const Geo& G, int e, int n3, int t) {
  const size_t nE = G.nElems;
  const bool el = ELEM && G.em[9 * nE + e] > 0.0;
  NodeMetric m;
  m.base = el ? G.em : G.Ja;
  m.off = el ? (size_t)e : (size_t)e * n3 + t;
  m.st = el ? nE : nE * n3;
  return m;
}

// Element of a one-element-per-workgroup launch.  Consecutive workgroups are
// dealt round-robin to the chip's 8 XCDs, each with its own L2.  With
// XCD-aware numbering (DGX_XCD_REMAP 1) XCD x walks a contiguous block of
// elements, so an element and its lexicographic neighbours (which read the
// same face data) run on the same XCD close in time.  XCD x then gets
// nE/8 (+1 for x < nE%8) elements starting at x (nE/8) + min(x, nE%8); the
// map is a bijection of [0, nE) for any nE.  Measured, it gains nothing at
// N = 7 and costs 2-8 % at N = 3 (plausibly because in plain order the
// eight XCDs work on neighbouring elements at the same time and share the
// face data through the chip-wide last-level cache), so plain order (0) is
// the default.
#ifndef DGX_XCD_REMAP
#define DGX_XCD_REMAP 0
#endif
__device__ __forceinline__ int elem_of_block(int bid, int nE) {
  if constexpr (DGX_XCD_REMAP) {
    constexpr int kXcd = 8;
    const int q = nE / kXcd, r = nE - q * kXcd;
    int x, slot;
    if (bid < kXcd * q) { x = bid % kXcd; slot = bid / kXcd; }
    else { x = bid - kXcd * q; slot = q; }
    return x * q + (x < r ? x : r) + slot;
  } else {
    return bid;
  }
}

__device__ __forceinline__ size_t tr_index(int slot, int v, int nvar, int nSides, int side, int n2, int fi) {
  return (((size_t)slot * nvar + v) * nSides + side) * n2 + fi;
}

// Entropy-projected traces (split form on Gauss nodes): their ln rho and
// ln beta sit behind the trace values, at Utr + 2 tnv nSides n2 (tnv values
// per face node: 5, or 10 in FV contexts), layout [slot][2][side][(p,q)].
__device__ __forceinline__ double* trace_logs(double* Utr, int nS, int n2, int tnv = 5) {
  return Utr + (size_t)2 * tnv * nS * n2;
}
__device__ __forceinline__ const double* trace_logs(const double* Utr, int nS, int n2, int tnv = 5) {
  return Utr + (size_t)2 * tnv * nS * n2;
}

}  // namespace dgx

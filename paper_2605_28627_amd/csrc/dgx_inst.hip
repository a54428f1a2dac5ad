// dgx_inst.hip -- launchers of the residual kernels for one polynomial degree.
// Compiled once per degree with -DDGX_INST_N=<N>; the launchers are named
// launch_*_N<N> and dispatched at run time by dgx_launch.hip.
#include "dgx_adjoint.hpp"
#include "dgx_kernels.hpp"

#ifndef DGX_INST_N
#error "DGX_INST_N must be defined"
#endif

#define DGX_CAT2(a, b) a##b
#define DGX_CAT(a, b) DGX_CAT2(a, b)
#define DGX_NAME(base) DGX_CAT(base, DGX_CAT(_N, DGX_INST_N))

namespace dgx {

constexpr int kN = DGX_INST_N;

hipError_t DGX_NAME(launch_trace)(const Cfg& c, const Geo& g, const Phys& p, const double* U, double* Utr,
                                  hipStream_t s) {
  const dim3 grid(g.nElems), block(Shape<kN>::nth);
  if (c.nodes == 1)
    hipLaunchKernelGGL((k_trace<kN, 1, 0>), grid, block, 0, s, g, p, U, Utr);
  else if (c.form == 0)
    hipLaunchKernelGGL((k_trace<kN, 0, 0>), grid, block, 0, s, g, p, U, Utr);
  else
    hipLaunchKernelGGL((k_trace<kN, 0, 1>), grid, block, 0, s, g, p, U, Utr);
  return hipGetLastError();
}

template <int NODES>
static void lift_emit(const Cfg& c, int emit, const Geo& g, const Phys& p, const double* U, const double* Utr,
                      double* gout, double* gtr, hipStream_t s) {
  const dim3 grid(g.nElems), block(Shape<kN>::nth);
  if (emit == 0)
    hipLaunchKernelGGL((k_lift<kN, NODES, 0, 0, 0>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
  else if (c.precision == 0 && c.visc == 0)
    hipLaunchKernelGGL((k_lift<kN, NODES, 1, 0, 0>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
  else if (c.precision == 0)
    hipLaunchKernelGGL((k_lift<kN, NODES, 1, 0, 1>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
  else if (c.visc == 0)
    hipLaunchKernelGGL((k_lift<kN, NODES, 1, 1, 0>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
  else
    hipLaunchKernelGGL((k_lift<kN, NODES, 1, 1, 1>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
}

hipError_t DGX_NAME(launch_lift)(const Cfg& c, int emit, const Geo& g, const Phys& p, const double* U,
                                 const double* Utr, double* gout, double* gtr, hipStream_t s) {
  if (c.fv) {
    // FV contexts (FP64, constant viscosity): DG elements without an FV face
    // (lean kernel), DG elements with one, then FV elements' Green-Gauss
    // gradients; the layer-0 gradients go behind the face fluxes
    const dim3 grid(g.nElems), block(Shape<kN>::nth);
    double* gtr2 = gtr + (size_t)8 * g.nSides * Shape<kN>::n2;
    if (emit != 1) return hipErrorInvalidValue;
    if (c.nodes == 1)
      hipLaunchKernelGGL((k_lift<kN, 1, 1, 0, 0, 3>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
    else
      hipLaunchKernelGGL((k_lift<kN, 0, 1, 0, 0, 3>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
    if (c.nodes == 1)
      hipLaunchKernelGGL((k_lift<kN, 1, 1, 0, 0, 1>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
    else if (c.form == 0)
      hipLaunchKernelGGL((k_lift<kN, 0, 1, 0, 0, 1>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
    else
      hipLaunchKernelGGL((k_lift<kN, 0, 1, 0, 0, 2>), grid, block, 0, s, g, p, U, Utr, gout, gtr);
    hipLaunchKernelGGL((k_lift_fv<kN>), grid, block, 0, s, g, p, U, Utr, gout, gtr2);
    return hipGetLastError();
  }
  if (c.nodes == 1)
    lift_emit<1>(c, emit, g, p, U, Utr, gout, gtr, s);
  else
    lift_emit<0>(c, emit, g, p, U, Utr, gout, gtr, s);
  return hipGetLastError();
}

template <int NODES, int FORM, int PHYS, int PREC, int ROE>
static void vol_mode_r(int mode, const Geo& g, const Phys& p, const double* U, const double* Utr, const double* gvn,
                       const double* gvf, double* Ut, double* Uio, double* dU, double* Utr_next, double A, double B,
                       double dt, hipStream_t s) {
  const dim3 grid(g.nElems), block(Shape<kN>::nth);
  if (mode == 0)
    hipLaunchKernelGGL((k_volume<kN, NODES, FORM, PHYS, PREC, 0, ROE>), grid, block, 0, s, g, p, U, Utr, gvn, gvf,
                       Ut, Uio, dU, Utr_next, A, B, dt);
  else
    hipLaunchKernelGGL((k_volume<kN, NODES, FORM, PHYS, PREC, 1, ROE>), grid, block, 0, s, g, p, U, Utr, gvn, gvf,
                       Ut, Uio, dU, Utr_next, A, B, dt);
}

template <int NODES, int FORM, int PHYS, int PREC>
static void vol_mode(int mode, int roe, const Geo& g, const Phys& p, const double* U, const double* Utr,
                     const double* gvn, const double* gvf, double* Ut, double* Uio, double* dU, double* Utr_next,
                     double A, double B, double dt, hipStream_t s) {
  if (roe)
    vol_mode_r<NODES, FORM, PHYS, PREC, 1>(mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  else
    vol_mode_r<NODES, FORM, PHYS, PREC, 0>(mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
}

template <int NODES, int FORM>
static void vol_phys(const Cfg& c, int mode, const Geo& g, const Phys& p, const double* U, const double* Utr,
                     const double* gvn, const double* gvf, double* Ut, double* Uio, double* dU, double* Utr_next,
                     double A, double B, double dt, hipStream_t s) {
  if (c.physics == 0) {
    if (c.precision == 0) vol_mode<NODES, FORM, 0, 0>(mode, c.roe, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
    else vol_mode<NODES, FORM, 0, 1>(mode, c.roe, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  } else {
    if (c.precision == 0) vol_mode<NODES, FORM, 1, 0>(mode, c.roe, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
    else vol_mode<NODES, FORM, 1, 1>(mode, c.roe, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  }
}

// DG elements of an FV context (FP64, Rusanov; Navier-Stokes with constant
// viscosity; the split form on Gauss nodes is the entropy-stable hybridised
// form).  Navier-Stokes: those without an FV face in the lean kernel (FV 2),
// then those with one (FV 1), each kernel skipping the other's elements (the
// FV-face variants need far more registers and LDS there); Euler: one kernel.
template <int NODES, int FORM, int PHYS>
static void vol_fv(int mode, const Geo& g, const Phys& p, const double* U, const double* Utr, const double* gvn,
                   const double* gvf, double* Ut, double* Uio, double* dU, double* Utr_next, double A, double B,
                   double dt, hipStream_t s) {
  const dim3 grid(g.nElems), block(Shape<kN>::nth);
  if (mode == 0) {
    if constexpr (PHYS == 1)
      hipLaunchKernelGGL((k_volume<kN, NODES, FORM, PHYS, 0, 0, 0, 2>), grid, block, 0, s, g, p, U, Utr, gvn, gvf,
                         Ut, Uio, dU, Utr_next, A, B, dt);
    hipLaunchKernelGGL((k_volume<kN, NODES, FORM, PHYS, 0, 0, 0, 1>), grid, block, 0, s, g, p, U, Utr, gvn, gvf,
                       Ut, Uio, dU, Utr_next, A, B, dt);
  } else {
    if constexpr (PHYS == 1)
      hipLaunchKernelGGL((k_volume<kN, NODES, FORM, PHYS, 0, 1, 0, 2>), grid, block, 0, s, g, p, U, Utr, gvn, gvf,
                         Ut, Uio, dU, Utr_next, A, B, dt);
    hipLaunchKernelGGL((k_volume<kN, NODES, FORM, PHYS, 0, 1, 0, 1>), grid, block, 0, s, g, p, U, Utr, gvn, gvf,
                       Ut, Uio, dU, Utr_next, A, B, dt);
  }
}

template <int PHYS>
static void vol_fv_form(const Cfg& c, int mode, const Geo& g, const Phys& p, const double* U, const double* Utr,
                        const double* gvn, const double* gvf, double* Ut, double* Uio, double* dU, double* Utr_next,
                        double A, double B, double dt, hipStream_t s) {
  if (c.nodes == 0 && c.form == 0) vol_fv<0, 0, PHYS>(mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  else if (c.nodes == 0) vol_fv<0, 1, PHYS>(mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  else if (c.form == 0) vol_fv<1, 0, PHYS>(mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  else vol_fv<1, 1, PHYS>(mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
}

hipError_t DGX_NAME(launch_volume)(const Cfg& c, const Geo& g, const Phys& p, int mode, const double* U,
                                   const double* Utr, const double* gvn, const double* gvf, double* Ut, double* Uio,
                                   double* dU, double* Utr_next, double A, double B, double dt, hipStream_t s) {
  if (c.fv) {
    if (c.physics == 0) vol_fv_form<0>(c, mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
    else vol_fv_form<1>(c, mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
    return hipGetLastError();
  }
  if (c.nodes == 0 && c.form == 0)
    vol_phys<0, 0>(c, mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  else if (c.nodes == 0)
    vol_phys<0, 1>(c, mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  else if (c.form == 0)
    vol_phys<1, 0>(c, mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  else
    vol_phys<1, 1>(c, mode, g, p, U, Utr, gvn, gvf, Ut, Uio, dU, Utr_next, A, B, dt, s);
  return hipGetLastError();
}

hipError_t DGX_NAME(launch_trace_fv)(const Cfg& c, const Geo& g, const Phys& p, const double* U, double* Utr,
                                     hipStream_t s) {
  const dim3 grid(g.nElems), block(Shape<kN>::nth);
  if (c.nodes == 1)
    hipLaunchKernelGGL((k_trace_fv<kN, 1>), grid, block, 0, s, g, p, U, Utr);
  else if (c.form == 0)
    hipLaunchKernelGGL((k_trace_fv<kN, 0>), grid, block, 0, s, g, p, U, Utr);
  else
    hipLaunchKernelGGL((k_trace_fv<kN, 0, 1>), grid, block, 0, s, g, p, U, Utr);
  return hipGetLastError();
}

hipError_t DGX_NAME(launch_fv)(const Cfg& c, const Geo& g, const Phys& p, int mode, const double* U,
                               const double* Utr, const double* gin, const double* gtr, double* Ut, double* Uio,
                               double* dU, double* Utr_next, double A, double B, double dt, hipStream_t s) {
  const dim3 grid(g.nElems), block(Shape<kN>::nth);
  if (c.physics == 1) {
    const double* gtr2 = gtr + (size_t)8 * g.nSides * Shape<kN>::n2;
    if (mode == 0)
      hipLaunchKernelGGL((k_fv<kN, 0, 1>), grid, block, 0, s, g, p, U, Utr, gin, gtr2, Ut, Uio, dU, Utr_next, A, B, dt);
    else
      hipLaunchKernelGGL((k_fv<kN, 1, 1>), grid, block, 0, s, g, p, U, Utr, gin, gtr2, Ut, Uio, dU, Utr_next, A, B, dt);
  } else {
    if (mode == 0)
      hipLaunchKernelGGL((k_fv<kN, 0, 0>), grid, block, 0, s, g, p, U, Utr, nullptr, nullptr, Ut, Uio, dU, Utr_next, A,
                         B, dt);
    else
      hipLaunchKernelGGL((k_fv<kN, 1, 0>), grid, block, 0, s, g, p, U, Utr, nullptr, nullptr, Ut, Uio, dU, Utr_next, A,
                         B, dt);
  }
  return hipGetLastError();
}

hipError_t DGX_NAME(launch_fv_indicator)(const Cfg& c, const Geo& g, const double* U, double* ind, hipStream_t s) {
  (void)c;
  hipLaunchKernelGGL((k_fv_indicator<kN>), dim3(g.nElems), dim3(Shape<kN>::nth), 0, s, g, U, ind);
  return hipGetLastError();
}

hipError_t DGX_NAME(launch_fv_switch)(const Cfg& c, const Geo& g, double* U, double* dU, const int* etype_new,
                                      int* etype, hipStream_t s) {
  (void)c;
  hipLaunchKernelGGL((k_fv_switch<kN>), dim3(g.nElems), dim3(Shape<kN>::nth), 0, s, g, U, dU, etype_new, etype);
  return hipGetLastError();
}

hipError_t DGX_NAME(launch_adjoint)(const Cfg& c, const Geo& g, const Phys& p, const double* U, const double* lam,
                                    const double* Utr, double* Lbar, const double* gin, const double* gtr,
                                    double* out, double* qbar, const AdjUpd& up, hipStream_t s) {
  // the fused RK update goes into the last kernel: the volume adjoint (Euler)
  // or the lifting adjoint (Navier-Stokes)
  const AdjUpd none{nullptr, nullptr, 0.0, 0.0, 0.0};
  const AdjUpd& upv = c.physics == 1 ? none : up;
  const dim3 grid(g.nElems), block(Shape<kN>::nth);
  // per-element surface adjoints (unless the previous stage's last kernel wrote them)
  if (!up.lbar_ready) {
    if (c.nodes == 1)
      hipLaunchKernelGGL((k_adj_trace<kN, 1>), grid, block, 0, s, g, lam, Lbar);
    else
      hipLaunchKernelGGL((k_adj_trace<kN, 0>), grid, block, 0, s, g, lam, Lbar);
  }
  // volume + surface adjoint
#define DGX_ADJ_V(NODES, FORM, PHYS, ROE, VL)                                                                  \
  hipLaunchKernelGGL((k_adj_volume<kN, NODES, FORM, PHYS, ROE, VL>), grid, block, 0, s, g, p, U, lam, Utr, Lbar, gin, \
                     gtr, out, qbar, upv)
  // (Sutherland's law only matters with viscous terms)
#define DGX_ADJ(NODES, FORM, PHYS)                                       \
  do {                                                                   \
    if (c.roe) {                                                         \
      if (PHYS == 1 && c.visc) DGX_ADJ_V(NODES, FORM, PHYS, 1, PHYS);     \
      else DGX_ADJ_V(NODES, FORM, PHYS, 1, 0);                           \
    } else {                                                             \
      if (PHYS == 1 && c.visc) DGX_ADJ_V(NODES, FORM, PHYS, 0, PHYS);     \
      else DGX_ADJ_V(NODES, FORM, PHYS, 0, 0);                           \
    }                                                                    \
  } while (0)
  if (c.nodes == 0 && c.form == 0) {
    if (c.physics == 0) DGX_ADJ(0, 0, 0); else DGX_ADJ(0, 0, 1);
  } else if (c.nodes == 0) {
    if (c.physics == 0) DGX_ADJ(0, 1, 0); else DGX_ADJ(0, 1, 1);
  } else if (c.form == 0) {
    if (c.physics == 0) DGX_ADJ(1, 0, 0); else DGX_ADJ(1, 0, 1);
  } else {
    if (c.physics == 0) DGX_ADJ(1, 1, 0); else DGX_ADJ(1, 1, 1);
  }
#undef DGX_ADJ
#undef DGX_ADJ_V
  if (c.physics == 1) {
    // lifting adjoint (its face values in qbar, written by the volume adjoint)
    if (c.nodes == 1)
      hipLaunchKernelGGL((k_adj_lift_volume<kN, 1>), grid, block, 0, s, g, p, U, Utr, qbar, out, up);
    else if (c.form == 1)
      hipLaunchKernelGGL((k_adj_lift_volume<kN, 0, 1>), grid, block, 0, s, g, p, U, Utr, qbar, out, up);
    else
      hipLaunchKernelGGL((k_adj_lift_volume<kN, 0>), grid, block, 0, s, g, p, U, Utr, qbar, out, up);
  }
  return hipGetLastError();
}

}  // namespace dgx

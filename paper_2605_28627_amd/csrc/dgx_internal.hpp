// dgx_internal.hpp -- internal types shared by the host runtime and the HIP
// kernels of the DGSEM residual library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace dgx {

// Largest polynomial degree with compiled kernels and the basis storage size.
constexpr int kMaxN = 7;
constexpr int kMaxN1 = kMaxN + 1;

// Device copy of the 1-D operators of one context (all FP64).
struct DevBasis {
  double w[kMaxN1];               // quadrature weights
  double winv[kMaxN1];            // 1 / w
  double Lm[kMaxN1], Lp[kMaxN1];  // l_j(-1), l_j(+1)
  double Dhat[kMaxN1 * kMaxN1];   // Dhat[a*n1+l] = (w_l / w_a) D_{l a}  (weak-form volume operator)
  double DS[kMaxN1 * kMaxN1];     // DS[a*n1+l] = 2 D_{a l} - e_N e_N^T / w_N + e_0 e_0^T / w_0  (split form)
  double D[kMaxN1 * kMaxN1];      // D[a*n1+l] = l_l'(x_a)
  // FV sub-cells (zero unless enabled)
  double Bs[kMaxN1 * kMaxN1];     // Bs[k*n1+i] = integral of l_i over sub-interval k of [-1,1]
  double Bsi[kMaxN1 * kMaxN1];    // inverse of Bs
  double Vli[kMaxN1 * kMaxN1];    // inverse of the orthonormal-Legendre Vandermonde V[i*n1+m] = P~_m(x_i)
};

// Per-element face table entry: side index, slot (0 master / 1 slave), orientation.
__host__ __device__ inline int efc_pack(int side, int slot, int orient) { return (side << 4) | (slot << 3) | orient; }
__host__ __device__ inline int efc_side(int v) { return v >> 4; }
__host__ __device__ inline int efc_slot(int v) { return (v >> 3) & 1; }
__host__ __device__ inline int efc_orient(int v) { return v & 7; }

// Slave face-local (pp,qq) -> master (p,q) under orientation o (inverse of the
// master->slave map: swap if bit 2, then reverse first if bit 0, second if bit 1).
__host__ __device__ inline void orient_to_master(int o, int N, int pp, int qq, int& p, int& q) {
  int a = (o & 1) ? N - pp : pp;
  int b = (o & 2) ? N - qq : qq;
  if (o & 4) { p = b; q = a; } else { p = a; q = b; }
}

// Physical constants and switches seen by the kernels.
struct Phys {
  double gamma, gm1, mu, lam, R, Rinv, Pr;  // lam = mu gamma R / ((gamma-1) Pr): heat conductivity
  double igm1;                          // 1 / (gamma - 1)
  double kappa;                         // gamma R / ((gamma-1) Pr): conductivity over viscosity
  double Tref, Ts;                      // Sutherland's law: reference temperature, S / Tref
  int riemann;                          // 0 Rusanov, 1 central part only, 2 Roe (Harten-Hyman fix)
  int twopoint;                         // 0 Chandrashekar, 1 flux average
  int visc_law;                         // 0 constant mu, 1 Sutherland
  // reference state of the FP32-flux mode (its fluxes round deviations from
  // it): pressure, 1/beta = 2 p0/rho0, total enthalpy gamma p0/(gamma-1);
  // all 0 = none
  double p0, ib0, h0;
};

// Everything a kernel needs about the discretisation.
struct Geo {
  int nElems, nSides;
  const double* Ja;      // [9][nElems][n3], followed by sJ
  const double* sJ;      // [nElems][n3] (= Ja + 9 nElems n3)
  // [10][nElems]: an element's metric terms when they are the same at all of
  // its nodes (affine elements): Ja^r_n at 3r+n, 1/J at 9; 1/J = 0 (the
  // sign test em[9][e] > 0) sends the element's kernels to Ja and sJ
  const double* em;
  const double* face;    // [4][nSides][n2]: unit normal (3), surface element
  const int* efc;        // [nElems][6]
  const DevBasis* basis;
  // FV sub-cells (null unless enabled)
  const int* etype;      // [nElems]: 0 DG, 1 FV
  const int* sidefv;     // [nSides]: 1 if either element of the side is FV
  const int* efv;        // [nElems]: bit f (0..5) the side of face f is FV, bit 6 the element is FV
  const double* fvV;     // [nElems][n3] sub-cell volumes
  const double* fvS;     // [3 r * 3 c][nElems][N][n2] interior sub-face vectors (+xi_r)
  const double* fvSb;    // [3 c][nSides][n2] master-outward element-face sub-face vectors
};

// Kernel-side workspace pointers.
struct Work {
  double* Utr[2];        // ping-pong U traces: [2 slots][5][nSides][n2]
  double* gtr;           // gradient traces:     [2 slots][12][nSides][n2]
  double* g;             // lifted gradients:    [12][nElems][n3]
  double* red;           // reduction partials
  int* flag;             // state-check flag
};

struct Cfg {
  int N, nodes, form, physics, precision;
  int fv;    // FV sub-cells enabled (traces of 10 values, FV kernels)
  int roe;   // Roe's face flux (its own kernel instantiations)
  int visc;  // viscosity law (0 constant, 1 Sutherland; its own lifting instantiations)
};

// Launchers (defined in the kernel translation units).  Each returns the
// result of hipGetLastError() after the launch.
// Face traces of U (entropy-projected for the split form on Gauss nodes).
hipError_t launch_trace(const Cfg& c, const Geo& g, const Phys& p, const double* U, double* Utr, hipStream_t s);
// BR1 lifting.  emit 0: gradients g [12][nE][n3] and their traces
// [2][12][nSides][n2].  emit 1: the viscous fluxes the residual needs,
// G~^r [4r+v][nE][n3] and the per-side face-normal fluxes [2][4][nSides][n2]
// (in the buffers of g and of the traces).
hipError_t launch_lift(const Cfg& c, int emit, const Geo& g, const Phys& p, const double* U, const double* Utr,
                       double* gout, double* gtr, hipStream_t s);
// mode 0: Ut = R(U).  mode 1: dU = A dU + dt R(U); U += B dU; traces of the new U -> Utr_next.
// Navier-Stokes: gvn, gvf are the viscous fluxes written by launch_lift(emit 1).
hipError_t launch_volume(const Cfg& c, const Geo& g, const Phys& p, int mode, const double* U, const double* Utr,
                         const double* gvn, const double* gvf, double* Ut, double* Uio, double* dU, double* Utr_next,
                         double A, double B, double dt, hipStream_t s);

// The reverse LSERK update of one stage, fused into the last adjoint kernel:
// with lamU set, that kernel applies lamU += dt a, lamdU = A lamdU + Bnext lamU
// to a = (dR/dU)^T lam (lam being lamdU) instead of storing a in out.
struct AdjUpd {
  double* lamU;
  double* lamdU;
  double dt, A, Bnext;
  // Navier-Stokes: the surface adjoint of the updated lamdU (the next stage's
  // lam) is written to Lnext by the same kernel (null: not wanted); with
  // lbar_ready the Lbar of this stage's lam was written that way and the
  // surface-adjoint kernel is skipped
  double* Lnext;
  int lbar_ready;
};

// out = (dR/dU)^T lam (or, with up.lamU, the fused update); Utr holds the
// traces of U, Lbar/qbar are scratch (Navier-Stokes: gin/gtr hold the
// forward lifted gradients and their traces, qbar [2][4][nSides][n2] takes
// the lifting adjoint's face values, and out is scratch too when the update
// is fused).
hipError_t launch_adjoint(const Cfg& c, const Geo& g, const Phys& p, const double* U, const double* lam,
                          const double* Utr, double* Lbar, const double* gin, const double* gtr, double* out,
                          double* qbar, const AdjUpd& up, hipStream_t s);
// FV sub-cells.  Traces of an FV context hold 10 values per face node: the DG
// trace (values 0..4) on DG faces; on FV faces the primitive means of the
// first (0..4) and second (5..9) sub-cell layers under the face.
hipError_t launch_trace_fv(const Cfg& c, const Geo& g, const Phys& p, const double* U, double* Utr, hipStream_t s);
// FV elements' residual (mode 0) or RK stage and next traces (mode 1).
// Navier-Stokes: gin holds the FV elements' sub-cell gradients [12][nElems][n3]
// and gtr the lifting's face data (the layer-0 gradients behind 8 nSides n2).
hipError_t launch_fv(const Cfg& c, const Geo& g, const Phys& p, int mode, const double* U, const double* Utr,
                     const double* gin, const double* gtr, double* Ut, double* Uio, double* dU, double* Utr_next,
                     double A, double B, double dt, hipStream_t s);
hipError_t launch_fv_indicator(const Cfg& c, const Geo& g, const double* U, double* ind, hipStream_t s);
// Converts U and dU (may be null) of the elements whose type in etype_new
// differs from etype, then sets etype = etype_new.
hipError_t launch_fv_switch(const Cfg& c, const Geo& g, double* U, double* dU, const int* etype_new, int* etype,
                            hipStream_t s);
hipError_t launch_fv_decide(int nElems, const double* ind, double lo, double hi, const int* etype, int* etype_new,
                            hipStream_t s);
hipError_t launch_fv_side_flags(int nSides, const int* side_elem, const int* etype, int* sidefv, hipStream_t s);
hipError_t launch_fv_elem_flags(int nElems, const int* efc, const int* sidefv, const int* etype, int* efv, hipStream_t s);
hipError_t launch_scale_copy(size_t n, const double* x, double* y, double a, hipStream_t s);
hipError_t launch_fill(double* x, size_t n, double v, hipStream_t s);
hipError_t launch_fill_int(int* x, size_t n, int v, hipStream_t s);
hipError_t launch_kinetic_energy(const Cfg& c, const Geo& g, const double* U, double* partial, double* out,
                                 double scale, hipStream_t s);
hipError_t launch_kinetic_energy_grad(const Cfg& c, const Geo& g, const double* U, double* grad, double cJ,
                                      hipStream_t s);
hipError_t launch_timestep(const Cfg& c, const Geo& g, const Phys& p, const double* U, double* partial,
                           double* out2, hipStream_t s);
hipError_t launch_check_state(const Cfg& c, const Geo& g, const Phys& p, const double* U, int* flag,
                              hipStream_t s);
int reduction_blocks();

// Size of the static device scratch of dg_rk_step_noalloc, and its device
// address on the current device (looked up on the first call per device).
constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
hipError_t static_scratch(void** ptr);

}  // namespace dgx

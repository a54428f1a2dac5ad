// dgx_launch.hip -- run-time dispatch over the polynomial degree and the
// auxiliary kernels (fills, reductions for E_k and the time step, state check).
#include <hip/hip_runtime.h>

#include <mutex>

#include "dgx_internal.hpp"
#include "dgx_pointwise.hpp"

namespace dgx {

// ---------------------------------------------------------------------------
// Static scratch for dg_rk_step_noalloc: a file-scope device array of
// kStaticScratchBytes, one copy per GPU, held until the process ends.  In
// host code `scratch` only names the symbol; its device address is looked up
// once per device (with that device current) and cached, and only that
// address is ever handed to kernels or runtime calls.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

#define DGX_DECL(n)                                                                                           \
  hipError_t launch_trace_N##n(const Cfg&, const Geo&, const Phys&, const double*, double*, hipStream_t);   \
  hipError_t launch_lift_N##n(const Cfg&, int, const Geo&, const Phys&, const double*, const double*,      \
                              double*, double*, hipStream_t);                                                 \
  hipError_t launch_volume_N##n(const Cfg&, const Geo&, const Phys&, int, const double*, const double*,      \
                                const double*, const double*, double*, double*, double*, double*, double,   \
                                double, double, hipStream_t);                                                  \
  hipError_t launch_adjoint_N##n(const Cfg&, const Geo&, const Phys&, const double*, const double*,          \
                                 const double*, double*, const double*, const double*, double*, double*,       \
                                 const AdjUpd&, hipStream_t);                                                   \
  hipError_t launch_trace_fv_N##n(const Cfg&, const Geo&, const Phys&, const double*, double*, hipStream_t);   \
  hipError_t launch_fv_N##n(const Cfg&, const Geo&, const Phys&, int, const double*, const double*,         \
                            const double*, const double*, double*, double*, double*, double*, double, double,  \
                            double, hipStream_t);                                                              \
  hipError_t launch_fv_indicator_N##n(const Cfg&, const Geo&, const double*, double*, hipStream_t);           \
  hipError_t launch_fv_switch_N##n(const Cfg&, const Geo&, double*, double*, const int*, int*, hipStream_t);
DGX_DECL(1)
DGX_DECL(2)
DGX_DECL(3)
DGX_DECL(4)
DGX_DECL(5)
DGX_DECL(6)
DGX_DECL(7)
#undef DGX_DECL

#define DGX_SWITCH(call)            \
  switch (c.N) {                    \
    case 1: return call##_N1 ARGS;  \
    case 2: return call##_N2 ARGS;  \
    case 3: return call##_N3 ARGS;  \
    case 4: return call##_N4 ARGS;  \
    case 5: return call##_N5 ARGS;  \
    case 6: return call##_N6 ARGS;  \
    case 7: return call##_N7 ARGS;  \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_trace(const Cfg& c, const Geo& g, const Phys& p, const double* U, double* Utr, hipStream_t s) {
#define ARGS (c, g, p, U, Utr, s)
  DGX_SWITCH(launch_trace)
#undef ARGS
}

hipError_t launch_trace_fv(const Cfg& c, const Geo& g, const Phys& p, const double* U, double* Utr, hipStream_t s) {
#define ARGS (c, g, p, U, Utr, s)
  DGX_SWITCH(launch_trace_fv)
#undef ARGS
}

hipError_t launch_fv(const Cfg& c, const Geo& g, const Phys& p, int mode, const double* U, const double* Utr,
                     const double* gin, const double* gtr, double* Ut, double* Uio, double* dU, double* Utr_next,
                     double A, double B, double dt, hipStream_t s) {
#define ARGS (c, g, p, mode, U, Utr, gin, gtr, Ut, Uio, dU, Utr_next, A, B, dt, s)
  DGX_SWITCH(launch_fv)
#undef ARGS
}

hipError_t launch_fv_indicator(const Cfg& c, const Geo& g, const double* U, double* ind, hipStream_t s) {
#define ARGS (c, g, U, ind, s)
  DGX_SWITCH(launch_fv_indicator)
#undef ARGS
}

hipError_t launch_fv_switch(const Cfg& c, const Geo& g, double* U, double* dU, const int* etype_new, int* etype,
                            hipStream_t s) {
#define ARGS (c, g, U, dU, etype_new, etype, s)
  DGX_SWITCH(launch_fv_switch)
#undef ARGS
}

// New element types from the indicator: FV above hi, DG below lo, else unchanged.
__global__ void k_fv_decide(int n, const double* __restrict__ ind, double lo, double hi, const int* __restrict__ et,
                            int* __restrict__ et_new) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double x = ind[e];
  et_new[e] = x > hi ? 1 : (x < lo ? 0 : et[e]);
}

// A side is an FV face if either of its elements is FV.
__global__ void k_fv_side_flags(int n, const int* __restrict__ side_elem, const int* __restrict__ et,
                                int* __restrict__ sidefv) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  sidefv[s] = (et[side_elem[2 * s]] | et[side_elem[2 * s + 1]]) ? 1 : 0;
}

// Per element: which of its faces are FV (bits 0..5) and whether it is FV (bit 6).
__global__ void k_fv_elem_flags(int n, const int* __restrict__ efc, const int* __restrict__ sidefv,
                                const int* __restrict__ et, int* __restrict__ efv) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  int m = et[e] ? 64 : 0;
  for (int f = 0; f < 6; ++f) m |= sidefv[efc_side(efc[e * 6 + f])] ? (1 << f) : 0;
  efv[e] = m;
}

hipError_t launch_fv_decide(int nElems, const double* ind, double lo, double hi, const int* etype, int* etype_new,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_fv_decide, dim3((nElems + 255) / 256), dim3(256), 0, s, nElems, ind, lo, hi, etype, etype_new);
  return hipGetLastError();
}

hipError_t launch_fv_elem_flags(int nElems, const int* efc, const int* sidefv, const int* etype, int* efv, hipStream_t s) {
  hipLaunchKernelGGL(k_fv_elem_flags, dim3((nElems + 255) / 256), dim3(256), 0, s, nElems, efc, sidefv, etype, efv);
  return hipGetLastError();
}

hipError_t launch_fv_side_flags(int nSides, const int* side_elem, const int* etype, int* sidefv, hipStream_t s) {
  hipLaunchKernelGGL(k_fv_side_flags, dim3((nSides + 255) / 256), dim3(256), 0, s, nSides, side_elem, etype, sidefv);
  return hipGetLastError();
}

hipError_t launch_lift(const Cfg& c, int emit, const Geo& g, const Phys& p, const double* U, const double* Utr,
                       double* gout, double* gtr, hipStream_t s) {
#define ARGS (c, emit, g, p, U, Utr, gout, gtr, s)
  DGX_SWITCH(launch_lift)
#undef ARGS
}

hipError_t launch_volume(const Cfg& c, const Geo& g, const Phys& p, int mode, const double* U, const double* Utr,
                         const double* gin, const double* gtr, double* Ut, double* Uio, double* dU, double* Utr_next,
                         double A, double B, double dt, hipStream_t s) {
#define ARGS (c, g, p, mode, U, Utr, gin, gtr, Ut, Uio, dU, Utr_next, A, B, dt, s)
  DGX_SWITCH(launch_volume)
#undef ARGS
}

hipError_t launch_adjoint(const Cfg& c, const Geo& g, const Phys& p, const double* U, const double* lam,
                          const double* Utr, double* Lbar, const double* gin, const double* gtr, double* out,
                          double* qbar, const AdjUpd& up, hipStream_t s) {
#define ARGS (c, g, p, U, lam, Utr, Lbar, gin, gtr, out, qbar, up, s)
  DGX_SWITCH(launch_adjoint)
#undef ARGS
}

// ---------------------------------------------------------------------------
// Auxiliary kernels (grid-stride loops over nodes).
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;
int reduction_blocks() { return kRedBlocks; }

__global__ void k_fill(double* x, size_t n, double v) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) x[t] = v;
}
__global__ void k_fill_int(int* x, size_t n, int v) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) x[t] = v;
}

// y = a x (the reverse LSERK sweep starts with lamdU = B_{S-1} lamU).
__global__ void k_scale_copy(size_t n, const double* __restrict__ x, double* __restrict__ y, double a) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
    y[t] = a * x[t];
}

static unsigned grid_for(size_t n) {
  size_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  return (unsigned)(nb ? nb : 1);
}

hipError_t launch_scale_copy(size_t n, const double* x, double* y, double a, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, s, n, x, y, a);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, size_t n, double v, hipStream_t s) {
  size_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_int(int* x, size_t n, int v, hipStream_t s) {
  size_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)nb), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

__device__ inline double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}
__device__ inline double block_max(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] = fmax(sh[t], sh[t + w]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Quadrature weight w_i w_j w_k of node t of an element.
__device__ inline double node_weight(const DevBasis* b, int n1, int t) {
  const int i = t % n1, j = (t / n1) % n1, k = t / (n1 * n1);
  return b->w[i] * b->w[j] * b->w[k];
}

// E_k partial sums: sum w J |m|^2 / rho per block (fixed order, deterministic).
__global__ void k_ek_partial(Geo G, int n1, const double* __restrict__ U, double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const int n3 = n1 * n1 * n1;
  const size_t nv = (size_t)G.nElems * n3;
  double acc = 0.0;
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < nv; x += (size_t)gridDim.x * blockDim.x) {
    const double rho = U[x], m0 = U[nv + x], m1 = U[2 * nv + x], m2 = U[3 * nv + x];
    const double wJ = node_weight(G.basis, n1, (int)(x % n3)) / G.sJ[x];
    acc += wJ * ((m0 * m0 + m1 * m1 + m2 * m2) / rho);
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
__global__ void k_sum_final(const double* __restrict__ partial, int n, double scale, double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int x = threadIdx.x; x < n; x += blockDim.x) acc += partial[x];
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = s * scale;
}

hipError_t launch_kinetic_energy(const Cfg& c, const Geo& g, const double* U, double* partial, double* out,
                                 double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_ek_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, s, g, c.N + 1, U, partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kRedThreads), 0, s, partial, kRedBlocks, scale, out);
  return hipGetLastError();
}

// grad = cJ * d/dU (w J |m|^2/rho): (-w J |m|^2/rho^2, 2 w J m/rho, 0)
__global__ void k_ek_grad(Geo G, int n1, const double* __restrict__ U, double* __restrict__ grad, double cJ) {
  const int n3 = n1 * n1 * n1;
  const size_t nv = (size_t)G.nElems * n3;
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < nv; x += (size_t)gridDim.x * blockDim.x) {
    const double rho = U[x], m0 = U[nv + x], m1 = U[2 * nv + x], m2 = U[3 * nv + x];
    const double c = cJ * node_weight(G.basis, n1, (int)(x % n3)) / G.sJ[x];
    const double ri = 1.0 / rho;
    grad[x] = -c * (m0 * m0 + m1 * m1 + m2 * m2) * ri * ri;
    grad[nv + x] = 2.0 * c * m0 * ri;
    grad[2 * nv + x] = 2.0 * c * m1 * ri;
    grad[3 * nv + x] = 2.0 * c * m2 * ri;
    grad[4 * nv + x] = 0.0;
  }
}

hipError_t launch_kinetic_energy_grad(const Cfg& c, const Geo& g, const double* U, double* grad, double cJ,
                                      hipStream_t s) {
  hipLaunchKernelGGL(k_ek_grad, dim3(kRedBlocks), dim3(256), 0, s, g, c.N + 1, U, grad, cJ);
  return hipGetLastError();
}

// Time-step maxima: advective sum_r (|Ja^r.u| + c |Ja^r|) / J and viscous
// (mu/rho) max(4/3, gamma/Pr) sum_r |Ja^r|^2 / J^2.
__global__ void k_dt_partial(Geo G, Phys P, double visc_fac, int n1, const double* __restrict__ U,
                             double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const int n3 = n1 * n1 * n1;
  const size_t nv = (size_t)G.nElems * n3;
  double ma = 0.0, mv = 0.0;
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < nv; x += (size_t)gridDim.x * blockDim.x) {
    const double rho = U[x];
    const double u0 = U[nv + x] / rho, u1 = U[2 * nv + x] / rho, u2 = U[3 * nv + x] / rho;
    const double p = P.gm1 * (U[4 * nv + x] - 0.5 * rho * (u0 * u0 + u1 * u1 + u2 * u2));
    const double c = sqrt(P.gamma * p / rho);
    const double sJ = G.sJ[x];
    double sa = 0.0, sv = 0.0;
    for (int r = 0; r < 3; ++r) {
      const double a0 = G.Ja[(size_t)(3 * r) * nv + x], a1 = G.Ja[(size_t)(3 * r + 1) * nv + x],
                   a2 = G.Ja[(size_t)(3 * r + 2) * nv + x];
      const double nrm2 = a0 * a0 + a1 * a1 + a2 * a2;
      sa += fabs(a0 * u0 + a1 * u1 + a2 * u2) + c * sqrt(nrm2);
      sv += nrm2;
    }
    ma = fmax(ma, sa * sJ);
    Prim q;
    q.rho = rho; q.u[0] = u0; q.u[1] = u1; q.u[2] = u2; q.p = p;
    mv = fmax(mv, visc_mu<double>(q, P) / rho * visc_fac * sv * sJ * sJ);
  }
  double a = block_max(ma, sh);
  double b = block_max(mv, sh);
  if (threadIdx.x == 0) { partial[2 * blockIdx.x] = a; partial[2 * blockIdx.x + 1] = b; }
}
__global__ void k_max2_final(const double* __restrict__ partial, int n, double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double a = 0.0, b = 0.0;
  for (int x = threadIdx.x; x < n; x += blockDim.x) { a = fmax(a, partial[2 * x]); b = fmax(b, partial[2 * x + 1]); }
  double ra = block_max(a, sh);
  double rb = block_max(b, sh);
  if (threadIdx.x == 0) { out[0] = ra; out[1] = rb; }
}

hipError_t launch_timestep(const Cfg& c, const Geo& g, const Phys& p, const double* U, double* partial, double* out2,
                           hipStream_t s) {
  const double visc_fac = fmax(4.0 / 3.0, p.gamma / p.Pr);
  hipLaunchKernelGGL(k_dt_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, s, g, p, visc_fac, c.N + 1, U, partial);
  hipLaunchKernelGGL(k_max2_final, dim3(1), dim3(kRedThreads), 0, s, partial, kRedBlocks, out2);
  return hipGetLastError();
}

// Sets *flag when any node has rho <= 0, p <= 0 or a non-finite conserved value.
__global__ void k_check(Geo G, Phys P, int n1, const double* __restrict__ U, int* flag) {
  const int n3 = n1 * n1 * n1;
  const size_t nv = (size_t)G.nElems * n3;
  int bad = 0;
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < nv; x += (size_t)gridDim.x * blockDim.x) {
    const double r = U[x], a = U[nv + x], b = U[2 * nv + x], c = U[3 * nv + x], E = U[4 * nv + x];
    const bool fin = isfinite(r) && isfinite(a) && isfinite(b) && isfinite(c) && isfinite(E);
    const double p = P.gm1 * (E - 0.5 * (a * a + b * b + c * c) / r);
    if (!fin || !(r > 0.0) || !(p > 0.0)) bad = 1;
  }
  if (bad) flag[0] = 1;   // every writer stores the same value
}

hipError_t launch_check_state(const Cfg& c, const Geo& g, const Phys& p, const double* U, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check, dim3(kRedBlocks), dim3(256), 0, s, g, p, c.N + 1, U, flag);
  return hipGetLastError();
}

}  // namespace dgx

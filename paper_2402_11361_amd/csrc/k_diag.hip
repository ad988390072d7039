// Flow diagnostics of the Taylor-Green study (Sec. 5.3, eq. C5321): the
// volume-averaged kinetic energy and the dissipation rate
//   E_k = (1/|Omega|) int 1/2 rho |v|^2,
//   eps = 2 mu_eff / |Omega| int rho |omega|^2 / 2,   omega = curl v,
// with v = m / rho and d_k v_j = (q_k[m_j] - v_j q_k[rho]) / rho from the
// gradient variable q (2D: omega = d_x v_y - d_y v_x), integrated with the
// element quadrature.  One workgroup (one wave) per element in a grid-stride
// loop: the element's nodal u and q go to LDS, each lane takes quadrature
// points; per-workgroup sums, then one fixed-order sum (deterministic).
#include "context.h"
#include <mutex>

namespace {

constexpr int DIAG_THREADS = 64;
constexpr int DIAG_MAX_BLOCKS = 65536;

template <int D>
__global__ void __launch_bounds__(DIAG_THREADS)
    k_flow_diag(MeshDev md, const double* __restrict__ q, const double* __restrict__ u, long long nel,
                double* __restrict__ partial) {
  constexpr int NS = D + 2, NF = (1 + D) * NS;  // fields: u components, then q (k, c)
  extern __shared__ double nodal[];             // [NF][A]
  const int tid = threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};  // kinetic energy, enstrophy (rho-weighted), volume
  for (long long el = blockIdx.x; el < nel; el += gridDim.x) {
    const int macro = md.elem_macro[el];
    const ClassDev& cd = class_of(md, macro);
    const int e = (int)(el - md.el_off[macro]);
    const int A = cd.A, N = cd.N, Q = cd.Q;
    const double* ui = u + md.u_off[macro];
    const double* qi = q + (size_t)D * md.u_off[macro];
    const int* en = cd.elem_nodes + (size_t)e * A;
    __syncthreads();  // the previous element's values are consumed
    for (int i = tid; i < NF * A; i += DIAG_THREADS) {
      const int f = i / A, a = i % A;
      nodal[i] = (f < NS) ? ui[(size_t)f * N + en[a]] : qi[(size_t)(f - NS) * N + en[a]];
    }
    __syncthreads();
    for (int qp = tid; qp < Q; qp += DIAG_THREADS) {
      const double* phi = cd.Phi + (size_t)qp * A;
      double val[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) val[f] = 0.0;
      for (int a = 0; a < A; ++a) {
        const double ph = phi[a];
#pragma unroll
        for (int f = 0; f < NF; ++f) val[f] += ph * nodal[f * A + a];
      }
      const double rho = val[0];
      double v[D], dv[D][D];  // dv[j][k] = d_k v_j
      double v2 = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) { v[j] = val[1 + j] / rho; v2 += v[j] * v[j]; }
#pragma unroll
      for (int j = 0; j < D; ++j)
#pragma unroll
        for (int k = 0; k < D; ++k) dv[j][k] = (val[NS + k * NS + j + 1] - v[j] * val[NS + k * NS]) / rho;
      double om2;
      if constexpr (D == 3) {
        const double w0 = dv[2][1] - dv[1][2], w1 = dv[0][2] - dv[2][0], w2 = dv[1][0] - dv[0][1];
        om2 = w0 * w0 + w1 * w1 + w2 * w2;
      } else {
        const double w2 = dv[1][0] - dv[0][1];
        om2 = w2 * w2;
      }
      const double wq = cd.W[qp];
      acc[0] += wq * 0.5 * rho * v2;
      acc[1] += wq * 0.5 * rho * om2;
      acc[2] += wq;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
    for (int off = 32; off > 0; off >>= 1) acc[i] += __shfl_xor(acc[i], off, 64);
  if (tid == 0)
#pragma unroll
    for (int i = 0; i < 3; ++i) partial[(size_t)blockIdx.x * 3 + i] = acc[i];
}

// out = (E_k, eps, |Omega|) from the per-workgroup sums, in a fixed order.
__global__ void __launch_bounds__(DIAG_THREADS)
    k_flow_diag_finish(const double* __restrict__ partial, int nblk, double mu_eff, double* __restrict__ out) {
  __shared__ double s[3][DIAG_THREADS];
  const int tid = threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int b = tid; b < nblk; b += DIAG_THREADS)
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] += partial[(size_t)b * 3 + i];
#pragma unroll
  for (int i = 0; i < 3; ++i) s[i][tid] = acc[i];
  __syncthreads();
  if (tid == 0) {
    double t[3] = {0.0, 0.0, 0.0};
    for (int w = 0; w < DIAG_THREADS; ++w)
#pragma unroll
      for (int i = 0; i < 3; ++i) t[i] += s[i][w];
    out[0] = t[0] / t[2];
    out[1] = 2.0 * mu_eff * t[1] / t[2];
    out[2] = t[2];
  }
}

}  // namespace

namespace {

hipError_t launch_diag(HdgContext& c, const double* q, const double* u, double* partial, double* out3_dev) {
  const long long nel = c.hm.el_off[c.hm.n_macros];
  const int nblk = (int)std::min<long long>(nel, DIAG_MAX_BLOCKS);
  if (nblk < 1) return hipErrorInvalidValue;
  const size_t shm = sizeof(double) * (size_t)(1 + c.hm.dim) * c.hm.ns * c.cd.A;  // one degree for every class
  if (c.hm.dim == 3)
    hipLaunchKernelGGL(k_flow_diag<3>, dim3(nblk), dim3(DIAG_THREADS), shm, c.stream, c.md, q, u, nel, partial);
  else
    hipLaunchKernelGGL(k_flow_diag<2>, dim3(nblk), dim3(DIAG_THREADS), shm, c.stream, c.md, q, u, nel, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_flow_diag_finish, dim3(1), dim3(DIAG_THREADS), 0, c.stream, partial, nblk, c.ph.mu / c.ph.Re_c,
                     out3_dev);
  return hipGetLastError();
}

// Scratch of the variant without allocation: the three results, then the
// per-workgroup partial sums (3 per workgroup, at most DIAG_MAX_BLOCKS
// workgroups whatever the mesh size: the grid-stride loop folds further
// elements into them).  Every call on a device shares that device's copy and
// overwrites all of it before reading it; calls that overlap on one device
// race.  In host code the array's name is not a device address: kernels get
// the address looked up once per device by diag_scratch_setup.
constexpr int DIAG_SCRATCH_OUT = 4;
constexpr long long DIAG_SCRATCH_DOUBLES = DIAG_SCRATCH_OUT + 3LL * DIAG_MAX_BLOCKS;
static __device__ __align__(256) double scratch[DIAG_SCRATCH_DOUBLES];

constexpr int DIAG_MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_ptr[DIAG_MAX_DEVICES] = {};

}  // namespace

// Called at context set-up with the context's device current: looks up this
// device's address of `scratch` once.
hipError_t diag_scratch_setup(int device) {
  if (device < 0 || device >= DIAG_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[device]) return hipSuccess;
  double* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  scratch_ptr[device] = ptr;
  return hipSuccess;
}

hipError_t launch_flow_diagnostics(HdgContext& c, const double* q, const double* u, double* out3_dev) {
  return launch_diag(c, q, u, c.ws.red /* 3 DIAG_MAX_BLOCKS doubles of the 2^20 reduction buffer */, out3_dev);
}

// The same kernels with the static scratch of c.device; *out3_dev receives
// the device address of the three results (inside the scratch).
hipError_t launch_flow_diagnostics_static(HdgContext& c, const double* q, const double* u, double** out3_dev,
                                          std::string& err) {
  double* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (c.device >= 0 && c.device < DIAG_MAX_DEVICES) ptr = scratch_ptr[c.device];
  }
  if (!ptr) {
    err = "static scratch of the device was not set up";
    return hipErrorNotInitialized;
  }
  const long long nel = c.hm.el_off[c.hm.n_macros];
  const long long nblk = std::min<long long>(nel, DIAG_MAX_BLOCKS);
  if (DIAG_SCRATCH_OUT + 3 * nblk > DIAG_SCRATCH_DOUBLES) {
    err = "partial sums exceed the static scratch";
    return hipErrorInvalidValue;
  }
  *out3_dev = ptr;
  return launch_diag(c, q, u, ptr + DIAG_SCRATCH_OUT, ptr);
}

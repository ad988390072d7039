// Local recovery (paper eq. Csc4a, then Csc4b; Algorithm 1 after the global
// solve).  After the elimination the top n_u rows of each macro's W hold
// [U | U12 | w] with U12 = L^{-1} P (-C) and w = L^{-1} P f, so
//     dU = S^{-1} (f + C duhat) = U^{-1} (w - U12 duhat_i)          (Csc4a)
//     dQ_k = A_qq^{-1}(-R_Q - A_qu dU - A_q,uh duhat)_k
//          = -M^{-1} R_Q,k - C_k dU + sum_s sign_s M_k^{-1}[:, end_s] (x) duhat_(k,s)   (Csc4b)
#include "context.h"
#include <algorithm>

namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int local_face(const ClassDev& cd, int r) {
  int lf = 0;
  while (lf + 1 < 2 * cd.dim && r >= cd.nf_off[lf + 1]) ++lf;
  return lf;
}

constexpr int BS_ROWS = 64;

// z = w - U12 duhat_i for rows [blockIdx.x * 64, +64) of one macro.
// W is the eliminated matrix in its storage type T (double or float); the
// recovery itself runs in FP64.
template <class T>
__global__ void __launch_bounds__(256) k_bs_rhs(MeshDev md, int m0, const T* __restrict__ Wm,
                                                const double* __restrict__ x, double* __restrict__ z) {
  extern __shared__ double xs[];
  const int macro = m0 + blockIdx.y;
  const ClassDev& cd = class_of(md, macro);
  const int nb = cd.n_b, nu = cd.n_u, d = cd.dim, ld = cd.ldw, n_cols = cd.n_cols;
  if (blockIdx.x * BS_ROWS >= nu) return;
  for (int s = threadIdx.x; s < nb; s += blockDim.x) {
    const int lf = local_face(cd, s);
    const int F = md.macro_face[(size_t)macro * 2 * d + lf];
    xs[s] = x[md.face_off[F] + (s - cd.nf_off[lf])];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* Wmac = Wm + md.w_off[macro];
  for (int rr = wave; rr < BS_ROWS; rr += 4) {
    const int r = blockIdx.x * BS_ROWS + rr;
    if (r >= nu) break;
    double s = 0.0;
    for (int c = lane; c < nb; c += 64) s += (double)Wmac[wtix(r, nu + c, ld)] * xs[c];
    s = wave_sum(s);
    if (lane == 0) z[md.u_off[macro] + r] = (double)Wmac[wtix(r, n_cols - 1, ld)] - s;
  }
}

// Backward substitution U du = z in place (z -> du), one workgroup per macro,
// blocks of 64 rows from the bottom.
template <class T>
__global__ void __launch_bounds__(256) k_bs_trsv(MeshDev md, int m0, const T* __restrict__ Wm,
                                                 double* __restrict__ du) {
  __shared__ double sU[BS_ROWS][BS_ROWS + 1];
  __shared__ double sz[BS_ROWS];
  const int macro = m0 + blockIdx.x;
  const ClassDev& cd = class_of(md, macro);
  const int nu = cd.n_u, ld = cd.ldw;
  const T* U = Wm + md.w_off[macro];
  double* x = du + md.u_off[macro];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nblk = (nu + BS_ROWS - 1) / BS_ROWS;
  for (int b = nblk - 1; b >= 0; --b) {
    const int i0 = b * BS_ROWS, i1 = min(nu, i0 + BS_ROWS), nr = i1 - i0;
    // z[i0:i1] -= U[i0:i1, i1:nu] x[i1:nu]
    for (int rr = wave; rr < nr; rr += 4) {
      const int r = i0 + rr;
      double s = 0.0;
      for (int c = i1 + lane; c < nu; c += 64) s += (double)U[wtix(r, c, ld)] * x[c];
      s = wave_sum(s);
      if (lane == 0) sz[rr] = x[r] - s;
    }
    for (int i = threadIdx.x; i < nr * nr; i += blockDim.x) {
      const int r = i / nr, c = i % nr;
      sU[r][c] = (double)U[wtix(i0 + r, i0 + c, ld)];
    }
    __syncthreads();
    if (wave == 0) {
      // lane j keeps x_j of the block in a register
      double xv = (lane < nr) ? sz[lane] : 0.0;
      for (int r = nr - 1; r >= 0; --r) {
        double s = (lane > r && lane < nr) ? sU[r][lane] * xv : 0.0;
        s = wave_sum(s);
        if (lane == r) xv = (xv - s) / sU[r][r];
      }
      if (lane < nr) x[i0 + lane] = xv;
    }
    __syncthreads();
  }
}

// dQ for one (macro, direction k, component c) field.
__global__ void k_bs_dq(MeshDev md, const double* __restrict__ RQt, const double* __restrict__ du,
                        const double* __restrict__ duhat, double* __restrict__ dq) {
  const int ns = md.ns, d = md.dim;
  const int macro = blockIdx.x / (d * ns), f = blockIdx.x % (d * ns);
  const ClassDev& cd = class_of(md, macro);
  const int N = cd.N, nm = cd.nmax1;
  const int k = f / ns, c = f % ns;
  const int nk = cd.n1[k];
  const int stride = (k == 0) ? 1 : (k == 1 ? cd.n1[0] : cd.n1[0] * cd.n1[1]);
  const double* Ck = cd.C1D + (size_t)k * nm * nm;
  const double* Mk = cd.Minv1D + (size_t)k * nm * nm;
  const double* u = du + md.u_off[macro] + (size_t)c * N;
  const int Fm = md.macro_face[(size_t)macro * 2 * d + 2 * k];
  const int Fp = md.macro_face[(size_t)macro * 2 * d + 2 * k + 1];
  const int nf = cd.nf_nodes[2 * k];
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int ik = (i / stride) % nk;
    const int base = i - ik * stride;
    double s = 0.0;
    for (int j = 0; j < nk; ++j) s += Ck[ik * nm + j] * u[base + j * stride];
    // tangential trace index of node i on the faces normal to k
    int jt = 0, mul = 1, t = i;
    int idx[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) { idx[a] = t % cd.n1[a]; t /= cd.n1[a]; }
    for (int a = 0; a < d; ++a) {
      if (a == k) continue;
      jt += idx[a] * mul;
      mul *= cd.n1[a];
    }
    const double hm = duhat[md.face_off[Fm] + (size_t)c * nf + jt];
    const double hp = duhat[md.face_off[Fp] + (size_t)c * nf + jt];
    const double face = -Mk[ik * nm + 0] * hm + Mk[ik * nm + nk - 1] * hp;
    const size_t o = (size_t)d * md.u_off[macro] + (size_t)(k * ns + c) * N + i;
    dq[o] = -RQt[o] - s + face;
  }
}

}  // namespace

// Macros [m0, m1) from their eliminated matrices in W.
static hipError_t backsolve_range(HdgContext& c, const double* duhat, double* du, int m0, int m1, int nu, int nb) {
  const int nm = m1 - m0;
  if (nm <= 0) return hipSuccess;
  const dim3 grid_rhs((nu + BS_ROWS - 1) / BS_ROWS, nm);
  if (c.cond_prec == 1) {
    const float* W32 = reinterpret_cast<const float*>(c.ws.Wm);
    hipLaunchKernelGGL(k_bs_rhs<float>, grid_rhs, dim3(256), (size_t)nb * sizeof(double), c.stream, c.md, m0, W32,
                       duhat, du);
    hipLaunchKernelGGL(k_bs_trsv<float>, dim3(nm), dim3(256), 0, c.stream, c.md, m0, W32, du);
  } else {
    hipLaunchKernelGGL(k_bs_rhs<double>, grid_rhs, dim3(256), (size_t)nb * sizeof(double), c.stream, c.md, m0, c.ws.Wm,
                       duhat, du);
    hipLaunchKernelGGL(k_bs_trsv<double>, dim3(nm), dim3(256), 0, c.stream, c.md, m0, c.ws.Wm, du);
  }
  return hipGetLastError();
}

// Unchunked: W still holds every macro's elimination.  Chunked: each chunk
// is formed and its S rows eliminated again (the trace rows are not needed),
// in the precision of the last condensation, then recovered.
hipError_t launch_backsolve(HdgContext& c, const double* duhat, double* dq, double* du) {
  int nu = 0, nb = 0;
  for (const HostClass& k : c.hcs) { nu = std::max(nu, k.n_u); nb = std::max(nb, k.n_b); }
  const int nm = c.hm.n_macros;
  hipError_t e;
  if (!c.hm.chunked()) {
    if ((e = backsolve_range(c, duhat, du, 0, nm, nu, nb)) != hipSuccess) return e;
  } else {
    for (int j = 0; j < c.hm.n_chunks(); ++j) {
      const int m0 = c.hm.chunk_first[j], m1 = c.hm.chunk_first[j + 1];
      if ((e = launch_form(c, c.cond_prec, m0, m1)) != hipSuccess) return e;
      if ((e = launch_lu(c, c.cond_prec, j, true)) != hipSuccess) return e;
      if ((e = backsolve_range(c, duhat, du, m0, m1, nu, nb)) != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_bs_dq, dim3(nm * c.cd.dim * c.cd.ns), dim3(256), 0, c.stream, c.md, c.ws.RQt, du, duhat, dq);
  return hipGetLastError();
}

// Local recovery (paper eq. Csc4a, then Csc4b; Algorithm 1 after the global
// solve).  After the elimination the top n_u rows of each macro's W hold
// [U | U12 | w] with U12 = L^{-1} P (-C) and w = L^{-1} P f, so
//     dU = S^{-1} (f + C duhat) = U^{-1} (w - U12 duhat_i)          (Csc4a)
//     dQ_k = A_qq^{-1}(-R_Q - A_qu dU - A_q,uh duhat)_k
//          = -M^{-1} R_Q,k - C_k dU + sum_s sign_s M_k^{-1}[:, end_s] (x) duhat_(k,s)   (Csc4b)
//
// After an FP32 condensation the factors carry FP32 rounding; the recovery
// then refines dU in FP64 (iterative refinement of the S-solve): with dQ from
// Csc4b, the u-rows of the Newton system (eq. C312) give the FP64 residual
//     r = -(R_U + A_uq dQ + A_uu dU + A_u,uh duhat) = f + C duhat - S dU
// from the FP64 element and sub-face blocks of the linearisation, and
// dU += U^{-1} L^{-1} P r with the FP32 factors, a fixed number of sweeps.
// The elimination stores L column pair by column pair (128 columns), each
// pair's columns in the row order reached at the end of that pair, so
// L^{-1} P is applied pair by pair: the pair's row swaps, then its unit-lower
// columns.
#include "context.h"
#include <algorithm>
#include <vector>

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

// z = column n_u of the S rows: L^{-1} P (f + C duhat) after the elimination
// of the recovery form (the right-hand side folded into that column).
template <class T>
__global__ void __launch_bounds__(256) k_bs_col(MeshDev md, int m0, const T* __restrict__ Wm, double* __restrict__ z) {
  const int macro = m0 + blockIdx.y;
  const ClassDev& cd = class_of(md, macro);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= cd.n_u) return;
  z[md.u_off[macro] + r] = (double)Wm[md.w_off[macro] + wtix(r, cd.n_u, cd.ldw)];
}

// Where the factors of macro's S are: its eliminated matrix in W, or (st_off
// non-null) its copy in the factor store (n_u x n_u, ld = n_u rounded up to 64).
template <class T>
__device__ __forceinline__ const T* factors_of(const MeshDev& md, const ClassDev& cd, int macro, const T* base,
                                               const long long* st_off, int& ld) {
  if (st_off) {
    ld = (cd.n_u + 63) / 64 * 64;
    return base + st_off[macro];
  }
  ld = cd.ldw;
  return base + md.w_off[macro];
}

// Copy of the LU factors of S (the top-left n_u x n_u of each eliminated
// matrix of macros [m0, m0 + gridDim.y)) from W (type TW) to the factor
// store (type TS), tile by tile (16 x 64 tiles, the store's ld = n_u rounded
// up to 64; the columns past n_u of the last tile column carry W's values,
// which the solves never read).
template <class TW, class TS>
__global__ void __launch_bounds__(256) k_store_factors(MeshDev md, int m0, const TW* __restrict__ Wm,
                                                       const long long* __restrict__ st_off, TS* __restrict__ Fst) {
  const int macro = m0 + blockIdx.y;
  const ClassDev& cd = class_of(md, macro);
  const int nu = cd.n_u, ldu = (nu + 63) / 64 * 64;
  const long long n = (long long)((nu + 15) / 16 * 16) * ldu;  // elements of the stored tiles
  const TW* W = Wm + md.w_off[macro];
  TS* F = Fst + st_off[macro];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    // i -> (tile row R, tile column Cb, element within the 16 x 64 tile)
    const long long R = i / (16LL * ldu), rem = i % (16LL * ldu);
    const int Cb = (int)(rem >> 10), e = (int)(rem & 1023);
    F[i] = (TS)W[R * 16 * (long long)cd.ldw + (long long)Cb * 1024 + e];
  }
}

// Sum over c < nb of row[c] * xb[c], row = the 64 entries of one row of a
// 16 x 64 tile (contiguous, 16-byte aligned, read as 16-byte vectors), xb in
// LDS.  Entries past nb are read but not used.
__device__ __forceinline__ double row_dot64(const float* __restrict__ row, const double* xb, int nb) {
  const float4* v = reinterpret_cast<const float4*>(row);
  float4 a[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) a[k] = v[k];
  double s = 0.0;
  if (nb == 64) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      s += (double)a[k].x * xb[4 * k] + (double)a[k].y * xb[4 * k + 1] + (double)a[k].z * xb[4 * k + 2] +
           (double)a[k].w * xb[4 * k + 3];
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const float e[4] = {a[k].x, a[k].y, a[k].z, a[k].w};
#pragma unroll
      for (int t = 0; t < 4; ++t) s += (4 * k + t < nb) ? (double)e[t] * xb[4 * k + t] : 0.0;
    }
  }
  return s;
}
__device__ __forceinline__ double row_dot64(const double* __restrict__ row, const double* xb, int nb) {
  const double2* v = reinterpret_cast<const double2*>(row);
  double s = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {  // two halves of 16 loads each
    double2 a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = v[16 * h + k];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int c = 32 * h + 2 * k;
      s += (c < nb ? a[k].x * xb[c] : 0.0) + (c + 1 < nb ? a[k].y * xb[c + 1] : 0.0);
    }
  }
  return s;
}

// Backward substitution U du = z in place (z -> du), one workgroup per macro:
// blocks of 64 rows from the bottom, each solved by one wave (column by
// column), then subtracted from the rows above it (a thread per row, the
// block's 64 columns of that row read as vectors); z staged in LDS.
template <class T>
__global__ void __launch_bounds__(256) k_bs_trsv(MeshDev md, int m0, const T* __restrict__ Wm,
                                                 double* __restrict__ du, const long long* __restrict__ st_off = nullptr) {
  extern __shared__ double xs[];  // n_u
  __shared__ double sU[BS_ROWS][BS_ROWS + 1];
  const int macro = m0 + blockIdx.x;
  const ClassDev& cd = class_of(md, macro);
  const int nu = cd.n_u;
  int ld;
  const T* U = factors_of(md, cd, macro, Wm, st_off, ld);
  double* x = du + md.u_off[macro];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < nu; i += blockDim.x) xs[i] = x[i];
  const int nblk = (nu + BS_ROWS - 1) / BS_ROWS;
  for (int b = nblk - 1; b >= 0; --b) {
    const int i0 = b * BS_ROWS, nr = min(nu, i0 + BS_ROWS) - i0;
    for (int i = tid; i < nr * nr; i += blockDim.x) {
      const int r = i / nr, c = i % nr;
      sU[r][c] = (double)U[wtix(i0 + r, i0 + c, ld)];
    }
    __syncthreads();
    if (wave == 0) {
      double zv = (lane < nr) ? xs[i0 + lane] : 0.0;
      for (int r = nr - 1; r >= 0; --r) {
        if (lane == r) zv /= sU[r][r];
        const double xr = __shfl(zv, r, 64);
        if (lane < r) zv -= sU[lane][r] * xr;
      }
      if (lane < nr) xs[i0 + lane] = zv;
    }
    __syncthreads();
    for (int i = tid; i < i0; i += blockDim.x) xs[i] -= row_dot64(U + wtix(i, i0, ld), xs + i0, nr);
    __syncthreads();
  }
  for (int i = tid; i < nu; i += blockDim.x) x[i] = xs[i];
}

// dQ for one (macro, direction k, component c) field, macros from m0.
__global__ void k_bs_dq(MeshDev md, int m0, const double* __restrict__ RQt, const double* __restrict__ du,
                        const double* __restrict__ duhat, double* __restrict__ dq) {
  const int ns = md.ns, d = md.dim;
  const int macro = m0 + blockIdx.x / (d * ns), f = blockIdx.x % (d * ns);
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

struct ResidPtrs {
  const double *AUU, *AUQ, *SUB, *RU;
  int nsA, dnsA, sub_stride, off_AUB;
};

// r = -(R_U + A_uq dQ + A_uu dU + A_u,uh duhat) on the u-nodes of macro
// m0 + blockIdx.y: one wave per macro node (its n_s component rows), the
// elements through the node in their fixed order (deterministic sums).
__global__ void __launch_bounds__(256) k_bs_resid(MeshDev md, int m0, ResidPtrs rp, const double* __restrict__ du,
                                                  const double* __restrict__ dq, const double* __restrict__ duhat,
                                                  double* __restrict__ r) {
  const int macro = m0 + blockIdx.y;
  const ClassDev& cd = class_of(md, macro);
  const int lane = threadIdx.x & 63;
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a >= cd.N) return;  // whole waves only; no barrier below
  const int ns = cd.ns, d = cd.dim, A = cd.A, T = cd.T, N = cd.N;
  const int nsA = rp.nsA, dnsA = rp.dnsA, nst = ns * T;
  const long long uo = md.u_off[macro];
  const double* dU = du + uo;
  const double* dQ = dq + (size_t)d * uo;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int ie = 0; ie < cd.node_ne[a]; ++ie) {
    const int e = cd.node_e[a * 8 + ie], ae = cd.node_a[a * 8 + ie];
    const long long el = md.el_off[macro] + e;
    const int* en = cd.elem_nodes + (size_t)e * A;
    for (int c = 0; c < ns; ++c) {
      const double* auu = rp.AUU + ((size_t)el * nsA + (size_t)(c * A + ae)) * nsA;
      const double* auq = rp.AUQ + ((size_t)el * nsA + (size_t)(c * A + ae)) * dnsA;
      double s = 0.0;
      for (int i = lane; i < nsA; i += 64) s += auu[i] * dU[(size_t)(i / A) * N + en[i % A]];
      for (int i = lane; i < dnsA; i += 64) s += auq[i] * dQ[(size_t)(i / A) * N + en[i % A]];
      acc[c] += s;
    }
    for (int lf2 = 0; lf2 < 2 * d; ++lf2) {
      const int sid = cd.elem_sub[(size_t)e * 2 * d + lf2];
      if (sid < 0) continue;
      const int ta = cd.finv[(size_t)lf2 * A + ae];
      if (ta < 0) continue;
      const int F = md.macro_face[(size_t)macro * 2 * d + lf2];
      const int nf2 = cd.nf_nodes[lf2];
      const double* xh = duhat + md.face_off[F];
      const double* aub = rp.SUB + ((size_t)md.sub_off[macro] + sid) * rp.sub_stride + rp.off_AUB;
      const int* tid = cd.sub_tid + (size_t)sid * T;
      for (int c = 0; c < ns; ++c) {
        double s = 0.0;
        for (int i = lane; i < nst; i += 64) s += aub[(size_t)(c * T + ta) * nst + i] * xh[(i / T) * nf2 + tid[i % T]];
        acc[c] += s;
      }
    }
  }
  for (int c = 0; c < ns; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) r[uo + (size_t)c * N + a] = -(rp.RU[uo + (size_t)c * N + a] + v);
  }
}

// r <- L^{-1} P r for macro m0 + blockIdx.x with the factors of its S rows in
// W or the factor store (storage type T): per column pair, its row swaps
// (ipiv, in column order) then its unit-lower columns in 64-column blocks,
// each solved by one wave and subtracted from the rows below it (a thread per
// row, as in k_bs_trsv); r staged in LDS (n_u doubles).
template <class T>
__global__ void __launch_bounds__(256) k_bs_fwd(MeshDev md, int m0, const T* __restrict__ Wm,
                                                const int* __restrict__ ipiv_all, double* __restrict__ r,
                                                const long long* __restrict__ st_off = nullptr) {
  extern __shared__ double rs[];
  __shared__ double sL[BS_ROWS][BS_ROWS + 1];
  const int macro = m0 + blockIdx.x;
  const ClassDev& cd = class_of(md, macro);
  const int nu = cd.n_u;
  int ld;
  const T* W = factors_of(md, cd, macro, Wm, st_off, ld);
  const int* ipiv = ipiv_all + md.ipiv_off[macro];
  double* x = r + md.u_off[macro];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < nu; i += blockDim.x) rs[i] = x[i];
  __syncthreads();
  for (int j0 = 0; j0 < nu; j0 += 2 * BS_ROWS) {
    const int jend = min(nu, j0 + 2 * BS_ROWS);
    if (tid == 0)
      for (int col = j0; col < jend; ++col) {
        const int p = ipiv[col];
        if (p != col) { const double t = rs[col]; rs[col] = rs[p]; rs[p] = t; }
      }
    __syncthreads();
    for (int b0 = j0; b0 < jend; b0 += BS_ROWS) {
      const int nb = min(BS_ROWS, jend - b0);
      for (int i = tid; i < nb * nb; i += blockDim.x) {
        const int rr = i / nb, cc = i % nb;
        sL[rr][cc] = (double)W[wtix(b0 + rr, b0 + cc, ld)];
      }
      __syncthreads();
      if (wave == 0) {
        double xv = (lane < nb) ? rs[b0 + lane] : 0.0;
        for (int cc = 0; cc < nb; ++cc) {
          const double xc = __shfl(xv, cc, 64);
          if (lane > cc && lane < nb) xv -= sL[lane][cc] * xc;
        }
        if (lane < nb) rs[b0 + lane] = xv;
      }
      __syncthreads();
      for (int i = b0 + nb + tid; i < nu; i += blockDim.x) rs[i] -= row_dot64(W + wtix(i, b0, ld), rs + b0, nb);
      __syncthreads();
    }
  }
  for (int i = tid; i < nu; i += blockDim.x) x[i] = rs[i];
}

__global__ void k_zero_range(long long n, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = 0.0;
}

__global__ void k_add_range(long long n, const double* __restrict__ x, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] += x[i];
}

}  // namespace

// FP64 refinement sweeps of the recovery after an FP32 condensation (each
// gains about the relative accuracy of the factors: ~1e-5 for FP32, ~1e-2
// after trailing updates with BF16 operands).
constexpr int BS_REFINE_SWEEPS = 2;
constexpr int BS_REFINE_SWEEPS_BF16 = 8;

// Sweeps of du += S^{-1} r with r = the residual of the u-rows of eq. C44
// (FP64, from the element blocks: dQ from du and duhat, then
// -(R_U + A_uu du + A_uq dQ + A_u,uh duhat)) and S^{-1} applied with the
// factors in W (st_off null) or in the factor store, of storage type T.
// Starting from du = 0 the first sweep is the solve itself.  The Krylov
// vectors are free during the recovery and hold r (n_u_tot doubles).
template <class T>
static void refine_range(HdgContext& c, const double* duhat, double* dq, double* du, int m0, int m1, int nu,
                         const T* F, const long long* st_off, int sweeps) {
  const int nm = m1 - m0;
  double* r = c.ws.kry;
  int nmax = 0;
  for (const HostClass& k : c.hcs) nmax = std::max(nmax, k.N);
  const ResidPtrs rp{c.ws.AUU, c.ws.AUQ, c.ws.SUB, c.ws.RU, c.nsA, c.dnsA, c.sub_stride, c.off_AUB};
  const long long u0 = c.hm.u_off[m0], nr = c.hm.u_off[m1] - u0;
  const int nblk = (int)std::min<long long>((nr + 255) / 256, 65536);
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    hipLaunchKernelGGL(k_bs_dq, dim3(nm * c.cd.dim * c.cd.ns), dim3(256), 0, c.stream, c.md, m0, c.ws.RQt, du, duhat,
                       dq);
    hipLaunchKernelGGL(k_bs_resid, dim3((nmax + 3) / 4, nm), dim3(256), 0, c.stream, c.md, m0, rp, du, dq, duhat, r);
    hipLaunchKernelGGL(k_bs_fwd<T>, dim3(nm), dim3(256), (size_t)nu * sizeof(double), c.stream, c.md, m0, F,
                       c.ws.ipiv, r, st_off);
    hipLaunchKernelGGL(k_bs_trsv<T>, dim3(nm), dim3(256), (size_t)nu * sizeof(double), c.stream, c.md, m0, F, r,
                       st_off);
    hipLaunchKernelGGL(k_add_range, dim3(nblk), dim3(256), 0, c.stream, nr, r + u0, du + u0);
  }
}

// Sweeps of the recovery from the factor store: the FP64 factors of an FP64
// condensation need the solve alone; FP32 factors (an FP32 store or an FP32
// condensation) precondition FP64 refinement, each sweep gaining about the
// FP32 rounding times the conditioning of S.
constexpr int BS_STORE_SWEEPS_FP64 = 1;
constexpr int BS_STORE_SWEEPS_FP32 = 3;

// Macros [m0, m1) from their eliminated matrices in W.
// rhs_in_w: W holds the eliminated recovery form (right-hand side in column
// n_u) instead of the condensation's [U | U12 | w].
static hipError_t backsolve_range(HdgContext& c, const double* duhat, double* dq, double* du, int m0, int m1, int nu,
                                  int nb, bool rhs_in_w) {
  const int nm = m1 - m0;
  if (nm <= 0) return hipSuccess;
  const dim3 grid_rhs((nu + BS_ROWS - 1) / BS_ROWS, nm);
  const dim3 grid_col((nu + 255) / 256, nm);
  if (c.cond_prec == 1) {
    const float* W32 = reinterpret_cast<const float*>(c.ws.Wm);
    if (rhs_in_w)
      hipLaunchKernelGGL(k_bs_col<float>, grid_col, dim3(256), 0, c.stream, c.md, m0, W32, du);
    else
      hipLaunchKernelGGL(k_bs_rhs<float>, grid_rhs, dim3(256), (size_t)nb * sizeof(double), c.stream, c.md, m0, W32,
                         duhat, du);
    hipLaunchKernelGGL(k_bs_trsv<float>, dim3(nm), dim3(256), (size_t)nu * sizeof(double), c.stream, c.md, m0, W32,
                       du, nullptr);
    // FP64 refinement against the u-rows' residual
    const int sweeps = (c.bf16_update && !rhs_in_w) ? BS_REFINE_SWEEPS_BF16 : BS_REFINE_SWEEPS;
    refine_range<float>(c, duhat, dq, du, m0, m1, nu, W32, nullptr, sweeps);
  } else {
    if (rhs_in_w)
      hipLaunchKernelGGL(k_bs_col<double>, grid_col, dim3(256), 0, c.stream, c.md, m0, c.ws.Wm, du);
    else
      hipLaunchKernelGGL(k_bs_rhs<double>, grid_rhs, dim3(256), (size_t)nb * sizeof(double), c.stream, c.md, m0,
                         c.ws.Wm, duhat, du);
    hipLaunchKernelGGL(k_bs_trsv<double>, dim3(nm), dim3(256), (size_t)nu * sizeof(double), c.stream, c.md, m0,
                       c.ws.Wm, du, nullptr);
  }
  return hipGetLastError();
}

// Unchunked: W still holds every macro's elimination.  Chunked: each chunk's
// S rows are formed again with the right-hand side f + C duhat folded into
// column n_u (the trace rows and the C columns are not needed) and
// eliminated, in the precision of the last condensation, then recovered;
// the chunks condensed last (one per slot of W), whose eliminations W still
// holds when nothing has written W since, are recovered first and from there,
// as if unchunked.  With two slots the next chunk is formed on the formation
// stream while the current one is eliminated and recovered.
hipError_t launch_backsolve(HdgContext& c, const double* duhat, double* dq, double* du) {
  int nu = 0, nb = 0;
  for (const HostClass& k : c.hcs) { nu = std::max(nu, k.n_u); nb = std::max(nb, k.n_b); }
  const int nm = c.hm.n_macros;
  hipError_t e;
  // the refinement's residual lives in the Krylov vectors
  if ((c.cond_prec == 1 || (c.store_valid && c.hm.store_chunks > 0)) &&
      c.n_u_tot > (long long)(2 * c.kry_restart_max + c.kry_inner_max + 8) * c.hm.n_glob)
    return hipErrorInvalidValue;
  if (!c.hm.chunked()) {
    if ((e = backsolve_range(c, duhat, dq, du, 0, nm, nu, nb, false)) != hipSuccess) return e;
  } else {
    const int nch = c.hm.n_chunks();
    std::vector<char> done(nch, 0);
    if (c.store_valid && c.hm.store_chunks > 0) {
      // the leading chunks from the factor store, from du = 0
      const int m1 = c.hm.chunk_first[c.hm.store_chunks];
      const long long nr = c.hm.u_off[m1];
      hipLaunchKernelGGL(k_zero_range, dim3((unsigned)std::min<long long>((nr + 255) / 256, 65536)), dim3(256), 0,
                         c.stream, nr, du);
      // the factors carry the precision of the condensation at best
      const int sweeps = c.bf16_update ? 1 + BS_REFINE_SWEEPS_BF16
                                       : ((c.cond_prec == 1 || c.hm.store_prec == 1) ? BS_STORE_SWEEPS_FP32
                                                                                     : BS_STORE_SWEEPS_FP64);
      if (c.hm.store_prec == 1)
        refine_range<float>(c, duhat, dq, du, 0, m1, nu, reinterpret_cast<const float*>(c.ws.Fst), c.st_off_dev,
                            sweeps);
      else
        refine_range<double>(c, duhat, dq, du, 0, m1, nu, c.ws.Fst, c.st_off_dev, sweeps);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      for (int j = 0; j < c.hm.store_chunks; ++j) done[j] = 1;
      if ((e = report_progress(c, "recovery: stored chunks", c.hm.store_chunks, nch)) != hipSuccess) return e;
    }
    for (int r : c.w_res)
      if (r >= 0 && r < nch && !done[r]) {
        if ((e = backsolve_range(c, duhat, dq, du, c.hm.chunk_first[r], c.hm.chunk_first[r + 1], nu, nb, false)) !=
            hipSuccess)
          return e;
        done[r] = 1;
      }
    std::vector<int> todo;
    for (int j = 0; j < nch; ++j)
      if (!done[j]) todo.push_back(j);
    if (!todo.empty()) c.forget_w();  // W now takes recovery forms
    if (c.hm.slots() < 2) {
      for (int j : todo) {
        const int m0 = c.hm.chunk_first[j], m1 = c.hm.chunk_first[j + 1];
        if ((e = launch_form(c, c.cond_prec, m0, m1, -1, duhat)) != hipSuccess) return e;
        if ((e = launch_lu(c, c.cond_prec, j, true, -1, true)) != hipSuccess) return e;
        if ((e = backsolve_range(c, duhat, dq, du, m0, m1, nu, nb, true)) != hipSuccess) return e;
        if ((e = report_progress(c, "recovery: chunk", j + 1, nch)) != hipSuccess) return e;
      }
    } else if (!todo.empty()) {
      if ((e = form_stream_ready(c)) != hipSuccess) return e;
      hipStream_t fs = c.form_stream;
      hipEvent_t* ev = c.form_events;  // [0] start, [1 + b] slot b formed, [3 + b] slot b free
      // duhat and the recoveries from the resident chunks (which read both slots) come first
      if ((e = hipEventRecord(ev[0], c.stream)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(fs, ev[0], 0)) != hipSuccess) return e;
      bool used[2] = {false, false};
      auto form = [&](int j) -> hipError_t {
        hipError_t r;
        const int b = j % 2;
        if (used[b] && (r = hipStreamWaitEvent(fs, ev[3 + b], 0)) != hipSuccess) return r;
        used[b] = true;
        if ((r = launch_form(c, c.cond_prec, c.hm.chunk_first[j], c.hm.chunk_first[j + 1], -1, duhat, fs)) !=
            hipSuccess)
          return r;
        return hipEventRecord(ev[1 + b], fs);
      };
      if ((e = form(todo[0])) != hipSuccess) return e;
      for (size_t t = 0; t < todo.size(); ++t) {
        const int j = todo[t], b = j % 2;
        // the next chunk is formed ahead when it goes to the other slot
        const bool ahead = t + 1 < todo.size() && todo[t + 1] % 2 != b;
        if (ahead && (e = form(todo[t + 1])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(c.stream, ev[1 + b], 0)) != hipSuccess) return e;
        if ((e = launch_lu(c, c.cond_prec, j, true, -1, true)) != hipSuccess) return e;
        const int m0 = c.hm.chunk_first[j], m1 = c.hm.chunk_first[j + 1];
        if ((e = backsolve_range(c, duhat, dq, du, m0, m1, nu, nb, true)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev[3 + b], c.stream)) != hipSuccess) return e;
        if ((e = report_progress(c, "recovery: chunk", j + 1, nch)) != hipSuccess) return e;
        if (t + 1 < todo.size() && !ahead && (e = form(todo[t + 1])) != hipSuccess) return e;
      }
    }
  }
  hipLaunchKernelGGL(k_bs_dq, dim3(nm * c.cd.dim * c.cd.ns), dim3(256), 0, c.stream, c.md, 0, c.ws.RQt, du, duhat, dq);
  return hipGetLastError();
}

// After the elimination of chunk j (condensation precision prec): the
// factors of S of its macros that the factor store keeps.
hipError_t launch_store_factors(HdgContext& c, int prec, int chunk) {
  if (chunk >= c.hm.store_chunks) return hipSuccess;
  const int m0 = c.hm.chunk_first[chunk], nmc = c.hm.chunk_first[chunk + 1] - m0;
  const dim3 grid(1024, (unsigned)nmc);
  if (prec == 1) {
    const float* W = reinterpret_cast<const float*>(c.ws.Wm);
    if (c.hm.store_prec == 1)
      hipLaunchKernelGGL((k_store_factors<float, float>), grid, dim3(256), 0, c.stream, c.md, m0, W, c.st_off_dev,
                         reinterpret_cast<float*>(c.ws.Fst));
    else
      hipLaunchKernelGGL((k_store_factors<float, double>), grid, dim3(256), 0, c.stream, c.md, m0, W, c.st_off_dev,
                         c.ws.Fst);
  } else {
    if (c.hm.store_prec == 1)
      hipLaunchKernelGGL((k_store_factors<double, float>), grid, dim3(256), 0, c.stream, c.md, m0, c.ws.Wm,
                         c.st_off_dev, reinterpret_cast<float*>(c.ws.Fst));
    else
      hipLaunchKernelGGL((k_store_factors<double, double>), grid, dim3(256), 0, c.stream, c.md, m0, c.ws.Wm,
                         c.st_off_dev, c.ws.Fst);
  }
  return hipGetLastError();
}

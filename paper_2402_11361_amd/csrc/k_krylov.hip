// Global trace operator and preconditioner (paper Algorithm 2, Sec. 4.2) and
// the vector kernels of the Krylov solvers.
//
// y = A-hat x = sum_i P_i^T A-hat^{T_i} P_i x is applied in two passes: per
// macro a gather of its 2d face segments of x into LDS and a GEMV with the
// condensed block (rows streamed from HBM, one row per wave-iteration, four
// rows in flight), then a deterministic two-sided face sum.  The
// preconditioner applies the inverse face blocks of A_uh,uh (one dense
// n_f x n_f GEMV per face).
#include "context.h"
#include <algorithm>

namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// macro-local trace index -> local face
__device__ __forceinline__ int local_face(const ClassDev& cd, int r) {
  int lf = 0;
  while (lf + 1 < 2 * cd.dim && r >= cd.nf_off[lf + 1]) ++lf;
  return lf;
}

// out[g] = sum over the (one or two) sides of face F(g) of src(side macro, local index):
//   tiled == 0: src = base[b_off[macro] + index] (per-macro trace vectors),
//   tiled == 1: src = entry (n_u + index, n_cols - 1) of the macro's tiled matrix
//               (b-hat^{T_i} in the last column of the eliminated W).
// accumulate != 0 adds to out instead of overwriting it.
template <class TB>
__global__ void k_face_gather_sum(MeshDev md, const TB* __restrict__ base, int tiled, double* __restrict__ out,
                                  int accumulate) {
  const int d = md.dim;
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < md.n_glob; g += (long long)gridDim.x * blockDim.x) {
    const int F = find_in(md.face_off, md.n_faces, g);
    const int r = (int)(g - md.face_off[F]);
    const int mm = md.face_minus[F], mp = md.face_plus[F];
    int k = 0;
    const int m0 = mm >= 0 ? mm : mp;
    for (int lf = 0; lf < 2 * d; ++lf)
      if (md.macro_face[(size_t)m0 * 2 * d + lf] == F) { k = lf / 2; break; }
    double s = 0.0;
    auto at = [&](int macro, int lf) -> double {
      const ClassDev& cd = class_of(md, macro);
      const int idx = cd.nf_off[lf] + r;
      if (!tiled) return (double)base[md.b_off[macro] + idx];
      return (double)base[md.w_off[macro] + wtix(cd.n_u + idx, cd.n_cols - 1, cd.ldw)];
    };
    if (mm >= 0) s += at(mm, 2 * k + 1);
    if (mp >= 0) s += at(mp, 2 * k);
    out[g] = accumulate ? out[g] + s : s;
  }
}

constexpr int APPLY_ROWS = 64;
constexpr int APPLY_RB = 8;  // rows per pass of a wave (APPLY_ROWS / 4 divisible by it)

// ypart[b_off[macro] + r] = (A-hat^{T_i} x_i)_r.  TILED: A-hat inside the
// macro's tiled augmented matrix at (n_u, n_u); otherwise the compact
// row-major copy at a32_off[macro].  blockIdx.x covers 64 rows (the grid is
// sized for the largest class; rows beyond the macro's n_b do nothing).
template <class TA, bool TILED>
__global__ void __launch_bounds__(256) k_apply_local(MeshDev md, const TA* __restrict__ Ab, const double* __restrict__ x,
                                                     double* __restrict__ ypart) {
  extern __shared__ double xs[];
  const int macro = blockIdx.y;
  const ClassDev& cd = class_of(md, macro);
  const int nb = cd.n_b;
  if (blockIdx.x * APPLY_ROWS >= nb) return;
  const int d = cd.dim;
  for (int s = threadIdx.x; s < nb; s += blockDim.x) {
    const int lf = local_face(cd, s);
    const int F = md.macro_face[(size_t)macro * 2 * d + lf];
    xs[s] = x[md.face_off[F] + (s - cd.nf_off[lf])];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = blockIdx.x * APPLY_ROWS + wave * (APPLY_ROWS / 4);
  const TA* Am = Ab + (TILED ? md.w_off[macro] : md.a32_off[macro]);
  const long long ld = TILED ? cd.ldw : nb;
  const int off = TILED ? cd.n_u : 0;
  // APPLY_RB rows at a time: that many independent row streams per lane
  for (int rr = 0; rr < APPLY_ROWS / 4; rr += APPLY_RB) {
    const int r = r0 + rr;
    double acc[APPLY_RB];
#pragma unroll
    for (int i = 0; i < APPLY_RB; ++i) acc[i] = 0.0;
    if (TILED) {
      int q[APPLY_RB];
#pragma unroll
      for (int i = 0; i < APPLY_RB; ++i) q[i] = off + min(r + i, nb - 1);
      for (int s = lane; s < nb; s += 64) {
        const double xv = xs[s];
#pragma unroll
        for (int i = 0; i < APPLY_RB; ++i) acc[i] += (double)Am[wtix(q[i], off + s, ld)] * xv;
      }
    } else {
      const TA* p[APPLY_RB];
#pragma unroll
      for (int i = 0; i < APPLY_RB; ++i) p[i] = Am + (size_t)min(r + i, nb - 1) * ld;
      for (int s = lane; s < nb; s += 64) {
        const double xv = xs[s];
#pragma unroll
        for (int i = 0; i < APPLY_RB; ++i) acc[i] += (double)p[i][s] * xv;
      }
    }
#pragma unroll
    for (int i = 0; i < APPLY_RB; ++i) acc[i] = wave_sum(acc[i]);
    if (lane == 0) {
      double* yp = ypart + md.b_off[macro];
#pragma unroll
      for (int i = 0; i < APPLY_RB; ++i)
        if (r + i < nb) yp[r + i] = acc[i];
    }
  }
}

// FW[F] = [[A_F, -I], [I, 0]] with A_F the face block of A_uh,uh summed over
// both macro sides (sub-face blocks scattered to face trace nodes).
__global__ void k_face_build(MeshDev md, const double* __restrict__ SUB, int sub_stride, int off_ABB,
                             double* __restrict__ FW, long long face_stride, int ldf) {
  const int F = blockIdx.x;
  const int nf = md.face_ndof[F];
  const int nn = nf / md.ns;
  double* M = FW + (size_t)md.face_slot[F] * face_stride;
  for (int i = threadIdx.x; i < 2 * nf * ldf; i += blockDim.x) {
    const int r = i / ldf, c = i % ldf;
    double v = 0.0;
    if (r < nf && c == nf + r) v = -1.0;
    if (r >= nf && c == r - nf) v = 1.0;
    M[wtix(r, c, ldf)] = v;
  }
  __syncthreads();
  const int d = md.dim;
  for (int side = 0; side < 2; ++side) {
    const int macro = side == 0 ? md.face_minus[F] : md.face_plus[F];
    if (macro < 0) continue;
    const ClassDev& cd = class_of(md, macro);
    const int T = cd.T, ns = cd.ns, nst = ns * T;
    int lf = -1;
    for (int l = 0; l < 2 * d; ++l)
      if (md.macro_face[(size_t)macro * 2 * d + l] == F && (l % 2) == (side == 0 ? 1 : 0)) { lf = l; break; }
    if (lf < 0) continue;
    for (int sid = 0; sid < cd.n_sub; ++sid) {
      if (cd.sub_lf[sid] != lf) continue;
      const double* abb = SUB + ((size_t)md.sub_off[macro] + sid) * sub_stride + off_ABB;
      const int* tid = cd.sub_tid + (size_t)sid * T;
      __syncthreads();
      for (int i = threadIdx.x; i < nst * nst; i += blockDim.x) {
        const int rr = i / nst, cc = i % nst;
        const int c = rr / T, t = rr % T, cp = cc / T, tp = cc % T;
        M[wtix(c * nn + tid[t], cp * nn + tid[tp], ldf)] += abb[i];
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_precond_apply(MeshDev md, const double* __restrict__ FW, long long face_stride,
                                                       int ldf, const double* __restrict__ x, double* __restrict__ y) {
  extern __shared__ double xs[];
  const int F = blockIdx.x;
  const int nf = md.face_ndof[F];
  const long long off = md.face_off[F];
  for (int i = threadIdx.x; i < nf; i += blockDim.x) xs[i] = x[off + i];
  __syncthreads();
  const double* Ai = FW + (size_t)md.face_slot[F] * face_stride;  // A^{-1} at (nf, nf) of the tiled block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = wave; r < nf; r += 4) {
    double s = 0.0;
    for (int c = lane; c < nf; c += 64) s += Ai[wtix(nf + r, nf + c, ldf)] * xs[c];
    s = wave_sum(s);
    if (lane == 0) y[off + r] = s;
  }
}

// BF16 storage of the inner operator: the upper 16 bits of an IEEE single,
// rounded to nearest (ties to even); widened exactly on load.
struct Bf16 {
  unsigned short v;
  __device__ __forceinline__ operator double() const { return (double)__uint_as_float((unsigned)v << 16); }
};

__device__ __forceinline__ unsigned short to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan unchanged
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// A16[a32_off[macro] + r n_b + c] = bf16(A-hat^{T_i}[r][c]) from the tiled
// eliminated matrices (FP64 or FP32 storage)
template <class TW>
__global__ void k_cast_ahat16(MeshDev md, const TW* __restrict__ W, unsigned short* __restrict__ out) {
  const long long total = md.a32_off[md.n_macros];
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < total; g += (long long)gridDim.x * blockDim.x) {
    const int macro = find_in(md.a32_off, md.n_macros, g);
    const ClassDev& cd = class_of(md, macro);
    const long long rc = g - md.a32_off[macro];
    const int r = (int)(rc / cd.n_b), c = (int)(rc % cd.n_b);
    out[g] = to_bf16((float)W[md.w_off[macro] + wtix(cd.n_u + r, cd.n_u + c, cd.ldw)]);
  }
}

// A32[a32_off[macro] + r n_b + c] = (float) A-hat^{T_i}[r][c]
__global__ void k_cast_ahat(MeshDev md, const double* __restrict__ W, float* __restrict__ out) {
  const long long total = md.a32_off[md.n_macros];
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < total; g += (long long)gridDim.x * blockDim.x) {
    const int macro = find_in(md.a32_off, md.n_macros, g);
    const ClassDev& cd = class_of(md, macro);
    const long long rc = g - md.a32_off[macro];
    const int r = (int)(rc / cd.n_b), c = (int)(rc % cd.n_b);
    out[g] = (float)W[md.w_off[macro] + wtix(cd.n_u + r, cd.n_u + c, cd.ldw)];
  }
}

// Chunked condensation: A-hat^{T_i} (rows and columns [n_u, n_u + n_b) of
// the eliminated matrix) to the compact row-major copy at a32_off[macro], and
// b-hat^{T_i} (last column, plus the FP64 g kept outside W by the FP32 path)
// to bloc.  One workgroup per (row band, macro of the chunk).
template <class T>
__global__ void k_extract(MeshDev md, int m0, const T* __restrict__ W, T* __restrict__ Ac,
                          const double* __restrict__ gloc, double* __restrict__ bloc) {
  const int macro = m0 + blockIdx.y;
  const ClassDev& cd = class_of(md, macro);
  const int nb = cd.n_b, nu = cd.n_u;
  const T* Wm = W + md.w_off[macro];
  T* A = Ac + md.a32_off[macro];
  for (int r = blockIdx.x; r < nb; r += gridDim.x) {
    for (int k = threadIdx.x; k < nb; k += blockDim.x) A[(size_t)r * nb + k] = Wm[wtix(nu + r, nu + k, cd.ldw)];
    if (threadIdx.x == 0) {
      const double b = (double)Wm[wtix(nu + r, cd.n_cols - 1, cd.ldw)];
      bloc[md.b_off[macro] + r] = gloc ? gloc[md.b_off[macro] + r] + b : b;
    }
  }
}

// ---- vector kernels -------------------------------------------------------
constexpr int VEC_BLOCKS = 512;

__global__ void k_multidot_partial(long long n, int k, const double* __restrict__ V, long long ldv,
                                   const double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    const double* v = V + (size_t)j * ldv;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
      s += v[i] * w[i];
    s = wave_sum(s);
    if (lane == 0) sh[wave][0] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * k + j] = sh[0][0] + sh[1][0] + sh[2][0] + sh[3][0];
    __syncthreads();
  }
}

__global__ void k_multidot_final(int nblk, int k, const double* __restrict__ partial, double* __restrict__ out) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += partial[(size_t)b * k + j];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[j] = s;
}

__global__ void k_multiaxpy(long long n, int k, const double* __restrict__ V, long long ldv,
                            const double* __restrict__ coef, double sign, double* __restrict__ w) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += coef[j] * V[(size_t)j * ldv + i];
    w[i] += sign * s;
  }
}

__global__ void k_lincomb(long long n, int k, const double* __restrict__ V, long long ldv, const double* __restrict__ coef,
                          double* __restrict__ y, int accumulate) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double s = accumulate ? y[i] : 0.0;
    for (int j = 0; j < k; ++j) s += coef[j] * V[(size_t)j * ldv + i];
    y[i] = s;
  }
}

__global__ void k_scale_copy(long long n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

__global__ void k_sub(long long n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = a[i] - b[i];
}

__global__ void k_axpy(long long n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

__global__ void k_zero_ints(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// ---- device-resident Krylov control (no host synchronisation per step) ------

// col[i * stride] = (pass ? col[i * stride] : 0) + coef[i], i < n
__global__ void k_accum_col(int n, const double* __restrict__ coef, double* __restrict__ col, int stride, int pass) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) col[(size_t)i * stride] = (pass ? col[(size_t)i * stride] : 0.0) + coef[i];
}

// h = sqrt(max(dot, 0)); inv = 1 / h (0 if h = 0)
__global__ void k_norm_finish(const double* __restrict__ dot, double* __restrict__ h_out, double* __restrict__ inv_out) {
  const double h = sqrt(fmax(0.0, dot[0]));
  if (h_out) h_out[0] = h;
  inv_out[0] = h > 0.0 ? 1.0 / h : 0.0;
}

__global__ void k_scale_dev(long long n, const double* __restrict__ a, const double* __restrict__ x, double* __restrict__ y) {
  const double s = a[0];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = s * x[i];
}

// Column j of the (m+1) x m Hessenberg H (row-major, ld m): apply the
// previous rotations, form the new one, rotate g; res[j] = |g[j+1]|.
__global__ void k_givens_step(int j, int m, double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
                              double* __restrict__ g, double* __restrict__ res) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < j; ++i) {
    const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
    H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
    H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
  const double rr = hypot(a, b);
  cs[j] = rr > 0 ? a / rr : 1.0;
  sn[j] = rr > 0 ? b / rr : 0.0;
  H[(size_t)j * m + j] = rr;
  H[(size_t)(j + 1) * m + j] = 0.0;
  const double g0 = g[j];
  g[j] = cs[j] * g0;
  g[j + 1] = -sn[j] * g0;
  res[j] = fabs(g[j + 1]);
}

// y = argmin || beta e1 - H y || for the (k+1) x k Hessenberg H (ld ldh) by
// Givens rotations and back substitution (a zero pivot gives y_i = 0).
__global__ void k_small_ls(int k, int ldh, const double* __restrict__ Hin, const double* __restrict__ beta,
                           double* __restrict__ y) {
  if (threadIdx.x != 0) return;
  double R[17 * 16], g[17], cs[16], sn[16];
  for (int i = 0; i <= k; ++i)  // entries below the subdiagonal are not stored
    for (int j = 0; j < k; ++j) R[i * k + j] = (i <= j + 1) ? Hin[(size_t)i * ldh + j] : 0.0;
  for (int i = 0; i <= k; ++i) g[i] = 0.0;
  g[0] = beta[0];
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < j; ++i) {
      const double a = R[i * k + j], b = R[(i + 1) * k + j];
      R[i * k + j] = cs[i] * a + sn[i] * b;
      R[(i + 1) * k + j] = -sn[i] * a + cs[i] * b;
    }
    const double a = R[j * k + j], b = R[(j + 1) * k + j];
    const double rr = hypot(a, b);
    cs[j] = rr > 0 ? a / rr : 1.0;
    sn[j] = rr > 0 ? b / rr : 0.0;
    R[j * k + j] = rr;
    R[(j + 1) * k + j] = 0.0;
    const double g0 = g[j];
    g[j] = cs[j] * g0;
    g[j + 1] = -sn[j] * g0;
  }
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= R[i * k + j] * y[j];
    y[i] = R[i * k + i] != 0.0 ? s / R[i * k + i] : 0.0;
  }
}

inline unsigned grid_for(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4096)); }

}  // namespace

// out = sum over the sides of every face of the per-macro trace vector `base`
// (offsets b_off)
hipError_t launch_face_sum(HdgContext& c, const double* base, double* out) {
  hipLaunchKernelGGL(k_face_gather_sum<double>, dim3(grid_for(c.md.n_glob)), dim3(256), 0, c.stream, c.md, base, 0, out,
                     0);
  return hipGetLastError();
}

hipError_t launch_zero_ints(hipStream_t s, int* p, int n) {
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_bhat(HdgContext& c, double* bhat, int prec) {
  if (c.hm.chunked()) return launch_face_sum(c, c.ws.bloc, bhat);  // k_extract filled bloc
  // b-hat^{T_i}: column n_cols - 1 of rows [n_u, n_u + n_b) of each tiled matrix
  if (prec == 1) {
    // FP64 g first, then the FP32 correction -D S^{-1} f on top
    hipError_t e = launch_face_sum(c, c.ws.gloc, bhat);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_face_gather_sum<float>, dim3(grid_for(c.md.n_glob)), dim3(256), 0, c.stream, c.md,
                       reinterpret_cast<const float*>(c.ws.Wm), 1, bhat, 1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_face_gather_sum<double>, dim3(grid_for(c.md.n_glob)), dim3(256), 0, c.stream, c.md, c.ws.Wm, 1,
                     bhat, 0);
  return hipGetLastError();
}

// prec: 0 the condensed operator itself; 1 its FP32 copy (made by
// launch_cast_ahat, FP64 condensation only); 2 its BF16 copy (launch_cast_ahat16).
hipError_t launch_apply(HdgContext& c, const double* x, double* y, int prec) {
  int nb = 0;
  for (const HostClass& k : c.hcs) nb = std::max(nb, k.n_b);
  dim3 grid((nb + APPLY_ROWS - 1) / APPLY_ROWS, c.hm.n_macros);
  const size_t shm = (size_t)nb * sizeof(double);
  if (!c.hm.chunked() && prec == 2 && c.have_a16) {
    hipLaunchKernelGGL((k_apply_local<Bf16, false>), grid, dim3(256), shm, c.stream, c.md,
                       reinterpret_cast<const Bf16*>(c.ws.A16), x, c.ws.ypart);
  } else if (c.hm.chunked()) {  // compact copy of every macro's A-hat
    if (c.cond_prec == 1)
      hipLaunchKernelGGL((k_apply_local<float, false>), grid, dim3(256), shm, c.stream, c.md,
                         reinterpret_cast<const float*>(c.ws.Ac), x, c.ws.ypart);
    else
      hipLaunchKernelGGL((k_apply_local<double, false>), grid, dim3(256), shm, c.stream, c.md, c.ws.Ac, x, c.ws.ypart);
  } else if (c.cond_prec == 1) {  // FP32 condensation: the operator itself is FP32
    hipLaunchKernelGGL((k_apply_local<float, true>), grid, dim3(256), shm, c.stream, c.md,
                       reinterpret_cast<const float*>(c.ws.Wm), x, c.ws.ypart);
  } else if (prec == 1 && c.have_a32) {
    hipLaunchKernelGGL((k_apply_local<float, false>), grid, dim3(256), shm, c.stream, c.md, c.ws.A32, x, c.ws.ypart);
  } else {
    hipLaunchKernelGGL((k_apply_local<double, true>), grid, dim3(256), shm, c.stream, c.md, c.ws.Wm, x, c.ws.ypart);
  }
  return launch_face_sum(c, c.ws.ypart, y);
}

template <class T>
hipError_t lu_eliminate(hipStream_t s, T* W, int batch, long long mat_stride, int ld, int n_piv, int n_rows,
                        int n_cols, int* ipiv, int ipiv_stride, int* status, T* scratch, LuTune tune,
                        hipStream_t s2, hipEvent_t evA, hipEvent_t evF);

hipError_t launch_face_precond(HdgContext& c) {
  const long long fs = c.fstride;
  hipLaunchKernelGGL(k_face_build, dim3(c.hm.n_faces), dim3(256), 0, c.stream, c.md, c.ws.SUB, c.sub_stride,
                     c.off_ABB, c.ws.FW, fs, c.ldf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // blocks are stored grouped by face size; one batched elimination per size
  for (const auto& g : c.hm.face_groups) {
    const int nf = g[0], s0 = g[1], cnt = g[2];
    e = lu_eliminate<double>(c.stream, c.ws.FW + (size_t)s0 * fs, cnt, fs, c.ldf, nf, 2 * nf, 2 * nf,
                             c.ws.fpiv + (size_t)s0 * c.nf_max, c.nf_max,
                             reinterpret_cast<int*>(c.ws.small) + c.hm.n_chunks() * c.hm.n_classes, c.ws.Uinv,
                             LuTune{}, nullptr, nullptr, nullptr);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_precond_apply(HdgContext& c, const double* x, double* y) {
  const long long fs = c.fstride;
  hipLaunchKernelGGL(k_precond_apply, dim3(c.hm.n_faces), dim3(256), (size_t)c.nf_max * sizeof(double), c.stream, c.md,
                     c.ws.FW, fs, c.ldf, x, y);
  return hipGetLastError();
}

hipError_t launch_extract(HdgContext& c, int prec, int chunk) {
  const int m0 = c.hm.chunk_first[chunk], nmc = c.hm.chunk_first[chunk + 1] - m0;
  int nb = 0;
  for (const HostClass& k : c.hcs) nb = std::max(nb, k.n_b);
  const dim3 grid((unsigned)std::min(nb, 1024), (unsigned)nmc);
  if (prec == 1)
    hipLaunchKernelGGL(k_extract<float>, grid, dim3(256), 0, c.stream, c.md, m0,
                       reinterpret_cast<const float*>(c.ws.Wm), reinterpret_cast<float*>(c.ws.Ac), c.ws.gloc,
                       c.ws.bloc);
  else
    hipLaunchKernelGGL(k_extract<double>, grid, dim3(256), 0, c.stream, c.md, m0, c.ws.Wm, c.ws.Ac,
                       static_cast<const double*>(nullptr), c.ws.bloc);
  return hipGetLastError();
}

hipError_t launch_cast_ahat16(HdgContext& c) {
  const long long total = c.hm.a32_off[c.hm.n_macros];
  if (c.cond_prec == 1)
    hipLaunchKernelGGL(k_cast_ahat16<float>, dim3(grid_for(total)), dim3(256), 0, c.stream, c.md,
                       reinterpret_cast<const float*>(c.ws.Wm), c.ws.A16);
  else
    hipLaunchKernelGGL(k_cast_ahat16<double>, dim3(grid_for(total)), dim3(256), 0, c.stream, c.md,
                       static_cast<const double*>(c.ws.Wm), c.ws.A16);
  return hipGetLastError();
}

hipError_t launch_cast_ahat(HdgContext& c) {
  const long long total = c.hm.a32_off[c.hm.n_macros];
  hipLaunchKernelGGL(k_cast_ahat, dim3(grid_for(total)), dim3(256), 0, c.stream, c.md, c.ws.Wm, c.ws.A32);
  return hipGetLastError();
}

hipError_t launch_multidot(hipStream_t s, long long n, int k, const double* V, long long ldv, const double* w,
                           double* partial, double* out) {
  hipLaunchKernelGGL(k_multidot_partial, dim3(VEC_BLOCKS), dim3(256), 0, s, n, k, V, ldv, w, partial);
  hipLaunchKernelGGL(k_multidot_final, dim3(k), dim3(64), 0, s, VEC_BLOCKS, k, partial, out);
  return hipGetLastError();
}

hipError_t launch_multiaxpy(hipStream_t s, long long n, int k, const double* V, long long ldv, const double* coef,
                            double sign, double* w) {
  hipLaunchKernelGGL(k_multiaxpy, dim3(grid_for(n)), dim3(256), 0, s, n, k, V, ldv, coef, sign, w);
  return hipGetLastError();
}

hipError_t launch_lincomb(hipStream_t s, long long n, int k, const double* V, long long ldv, const double* coef,
                          double* y, int accumulate) {
  hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(256), 0, s, n, k, V, ldv, coef, y, accumulate);
  return hipGetLastError();
}

hipError_t launch_scale_copy(hipStream_t s, long long n, double a, const double* x, double* y) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_sub(hipStream_t s, long long n, const double* a, const double* b, double* y) {
  hipLaunchKernelGGL(k_sub, dim3(grid_for(n)), dim3(256), 0, s, n, a, b, y);
  return hipGetLastError();
}

hipError_t launch_axpy(hipStream_t s, size_t n, double a, const double* x, double* y) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for((long long)n)), dim3(256), 0, s, (long long)n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_accum_col(hipStream_t s, int n, const double* coef, double* col, int stride, int pass) {
  hipLaunchKernelGGL(k_accum_col, dim3(1), dim3(64), 0, s, n, coef, col, stride, pass);
  return hipGetLastError();
}

hipError_t launch_norm_finish(hipStream_t s, const double* dot, double* h_out, double* inv_out) {
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(1), 0, s, dot, h_out, inv_out);
  return hipGetLastError();
}

hipError_t launch_scale_dev(hipStream_t s, long long n, const double* a, const double* x, double* y) {
  hipLaunchKernelGGL(k_scale_dev, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_givens_step(hipStream_t s, int j, int m, double* H, double* cs, double* sn, double* g, double* res) {
  hipLaunchKernelGGL(k_givens_step, dim3(1), dim3(64), 0, s, j, m, H, cs, sn, g, res);
  return hipGetLastError();
}

hipError_t launch_small_ls(hipStream_t s, int k, int ldh, const double* Hin, const double* beta, double* y) {
  if (k > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_small_ls, dim3(1), dim3(64), 0, s, k, ldh, Hin, beta, y);
  return hipGetLastError();
}

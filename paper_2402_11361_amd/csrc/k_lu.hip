// Batched partial elimination with partial pivoting (blocked right-looking LU)
// of the augmented macro matrices W = [[S, -C, f], [D, E, g]] (paper eq. ASC2:
// S is factored, never inverted, remark after Csc4).
//
// Only the first n_piv columns are eliminated and pivots are searched only in
// the first n_piv rows (the S rows); the remaining rows (D, E, g) are
// eliminated without pivoting.  Afterwards
//   rows [0, n_piv):  U | L^{-1} P (-C) | L^{-1} P f     (used by the recovery)
//   rows [n_piv, .):  *  | E + D S^{-1} C | g - D S^{-1} f = A-hat^{T_i} | b-hat^{T_i}
// The same kernels invert the face blocks of A_uh,uh for the preconditioner
// ([[A, -I], [I, 0]] -> A^{-1} in the bottom-right corner).
//
// Per block of NB columns:
//   k_panel   one workgroup per matrix factors the S rows of the block in
//             sub-panels of PW columns held in registers (pivot search by a
//             workgroup arg-max, first maximum wins as in LAPACK);
//   k_dtrsm   L of the non-pivot rows: A_D,block U11^{-1};
//   k_update  one workgroup per (matrix, 64-column strip): row swaps, the
//             strip of U12 = L11^{-1} A12, and A22 -= L21 U12 on FP64 MFMA
//             (v_mfma_f64_16x16x4f64).
#include "context.h"

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int NB = 64;     // block width of the trailing update
constexpr int PW = 16;     // sub-panel width held in registers
constexpr int PANEL_THREADS = 512;
constexpr int NC = 64;     // strip width of the trailing update

struct LuArgs {
  double* W;
  long long mat_stride;  // doubles between matrices
  int ld, n_piv, n_rows, n_cols;
  int* ipiv;             // [batch][n_piv]
  int ipiv_stride;
  int* status;           // first singular matrix index + 1 (0 = none)
};

__device__ __forceinline__ void argmax_update(double& bv, int& bi, double v, int i) {
  if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
}

template <int RPT>
__global__ void __launch_bounds__(PANEL_THREADS) k_panel(LuArgs a, int j0, int jb) {
  const int tid = threadIdx.x;
  const int mat = blockIdx.x;
  double* W = a.W + (size_t)mat * a.mat_stride;
  int* ipiv = a.ipiv + (size_t)mat * a.ipiv_stride;
  const int ld = a.ld, n_piv = a.n_piv;
  __shared__ double s_bv[PANEL_THREADS / 64];
  __shared__ int s_bi[PANEL_THREADS / 64];
  __shared__ int s_prow;
  __shared__ double s_urow[PW];
  __shared__ double s_swap[2][PW];
  __shared__ double s_U[PW * NB];
  for (int c0 = j0; c0 < j0 + jb; c0 += PW) {
    const int pw = min(PW, j0 + jb - c0);
    // rows owned by this thread: c0 + tid + i * PANEL_THREADS
    double v[RPT][PW];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = c0 + tid + i * PANEL_THREADS;
#pragma unroll
      for (int cc = 0; cc < PW; ++cc) v[i][cc] = (r < n_piv && cc < pw) ? W[(size_t)r * ld + c0 + cc] : 0.0;
    }
    for (int cc = 0; cc < pw; ++cc) {
      {
      const int col = c0 + cc;
      // pivot search over rows [col, n_piv)
      double bv = -1.0;
      int bi = 0x7fffffff;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + i * PANEL_THREADS;
        double vc = v[i][0];
#pragma unroll
        for (int k = 1; k < PW; ++k) vc = (k == cc) ? v[i][k] : vc;
        if (r >= col && r < n_piv) argmax_update(bv, bi, fabs(vc), r);
      }
      for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(bv, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        argmax_update(bv, bi, ov, oi);
      }
      if ((tid & 63) == 0) { s_bv[tid >> 6] = bv; s_bi[tid >> 6] = bi; }
      __syncthreads();
      if (tid == 0) {
        double b = s_bv[0];
        int bi0 = s_bi[0];
        for (int w = 1; w < PANEL_THREADS / 64; ++w) argmax_update(b, bi0, s_bv[w], s_bi[w]);
        if (!(b > 0.0)) {  // zero or NaN column: singular
          if (a.status) atomicCAS(a.status, 0, mat + 1);
          bi0 = col;
        }
        s_prow = bi0;
        ipiv[col] = bi0;
      }
      __syncthreads();
      const int prow = s_prow;
      // exchange rows col and prow inside the sub-panel registers
      const int oc = col - c0, op = prow - c0;
      if (prow != col) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int rl = tid + i * PANEL_THREADS;
          if (rl == oc) {
#pragma unroll
            for (int k = 0; k < PW; ++k) s_swap[0][k] = v[i][k];
          }
          if (rl == op) {
#pragma unroll
            for (int k = 0; k < PW; ++k) s_swap[1][k] = v[i][k];
          }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int rl = tid + i * PANEL_THREADS;
          if (rl == oc) {
#pragma unroll
            for (int k = 0; k < PW; ++k) v[i][k] = s_swap[1][k];
          }
          if (rl == op) {
#pragma unroll
            for (int k = 0; k < PW; ++k) v[i][k] = s_swap[0][k];
          }
        }
        // the rest of the block row (columns [j0, c0) and [c0 + pw, j0 + jb)) in memory
        for (int k = tid; k < jb; k += PANEL_THREADS) {
          const int cidx = j0 + k;
          if (cidx >= c0 && cidx < c0 + pw) continue;
          double t = W[(size_t)col * ld + cidx];
          W[(size_t)col * ld + cidx] = W[(size_t)prow * ld + cidx];
          W[(size_t)prow * ld + cidx] = t;
        }
      }
      // broadcast the pivot row
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (tid + i * PANEL_THREADS == oc) {
#pragma unroll
          for (int k = 0; k < PW; ++k) s_urow[k] = v[i][k];
        }
      }
      __syncthreads();
      const double piv = s_urow[cc];
      const double ipv = (piv != 0.0) ? 1.0 / piv : 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + i * PANEL_THREADS;
        if (r > col && r < n_piv) {
          double vc = v[i][0];
#pragma unroll
          for (int k = 1; k < PW; ++k) vc = (k == cc) ? v[i][k] : vc;
          const double l = vc * ipv;
#pragma unroll
          for (int k = 0; k < PW; ++k) {
            if (k == cc) v[i][k] = l;
            if (k > cc) v[i][k] -= l * s_urow[k];
          }
        }
      }
      __syncthreads();
      }
    }
    // write the factored sub-panel back
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = c0 + tid + i * PANEL_THREADS;
      if (r < n_piv) {
#pragma unroll
        for (int cc = 0; cc < PW; ++cc)
          if (cc < pw) W[(size_t)r * ld + c0 + cc] = v[i][cc];
      }
    }
    // right-looking update of the rest of the block: columns [c0 + pw, j0 + jb)
    const int rest0 = c0 + pw, nrest = j0 + jb - rest0;
    __syncthreads();
    if (nrest > 0) {
      // U rows of the sub-panel: L_sub^{-1} A[c0:c0+pw, rest]  (unit lower, sequential rows)
      for (int k = tid; k < nrest; k += PANEL_THREADS) {
        for (int i = 0; i < pw; ++i) {
          double s = W[(size_t)(c0 + i) * ld + rest0 + k];
          for (int m = 0; m < i; ++m) s -= W[(size_t)(c0 + i) * ld + c0 + m] * s_U[m * NB + k];
          s_U[i * NB + k] = s;
        }
      }
      __syncthreads();
      for (int k = tid; k < pw * nrest; k += PANEL_THREADS) {
        const int i = k / nrest, cidx = k % nrest;
        W[(size_t)(c0 + i) * ld + rest0 + cidx] = s_U[i * NB + cidx];
      }
      // rows below the sub-panel: A[r, rest] -= L[r, c0:c0+pw] U
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + i * PANEL_THREADS;
        if (r >= c0 + pw && r < n_piv) {
          for (int cidx = 0; cidx < nrest; ++cidx) {
            double s = W[(size_t)r * ld + rest0 + cidx];
#pragma unroll
            for (int m = 0; m < PW; ++m)
              if (m < pw) s -= v[i][m] * s_U[m * NB + cidx];
            W[(size_t)r * ld + rest0 + cidx] = s;
          }
        }
      }
      __syncthreads();
    }
  }
}

// L of the non-pivot rows [n_piv, n_rows) for the block: l = a U11^{-1}.
// The workgroup first inverts the (identity-padded) upper triangle U11 in
// LDS, column by column; every thread then multiplies one row by it.
__global__ void __launch_bounds__(256) k_dtrsm(LuArgs a, int j0, int jb) {
  const int mat = blockIdx.y;
  double* W = a.W + (size_t)mat * a.mat_stride;
  const int ld = a.ld;
  __shared__ double sU[NB * NB];
  __shared__ double sI[NB * NB];
  for (int i = threadIdx.x; i < NB * NB; i += blockDim.x) {
    const int r = i / NB, c = i % NB;
    double v = (r == c) ? 1.0 : 0.0;
    if (r < jb && c < jb) v = W[(size_t)(j0 + r) * ld + j0 + c];
    sU[i] = v;
  }
  __syncthreads();
  if (threadIdx.x < NB) {
    const int j = threadIdx.x;  // column j of U^{-1}: U x = e_j, x_i = 0 for i > j
    for (int i = NB - 1; i >= 0; --i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int m = i + 1; m <= j; ++m) s -= sU[i * NB + m] * sI[m * NB + j];
      const double dgl = sU[i * NB + i];
      sI[i * NB + j] = (i <= j && dgl != 0.0) ? s / dgl : 0.0;
    }
  }
  __syncthreads();
  const int r = a.n_piv + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n_rows) return;
  double av[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) av[c] = (c < jb) ? W[(size_t)r * ld + j0 + c] : 0.0;
  for (int c = 0; c < jb; ++c) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < NB; ++m) s += av[m] * sI[m * NB + c];
    W[(size_t)r * ld + j0 + c] = s;
  }
}

// Trailing update of one 64-column strip to the right of the block.  Strips
// are aligned to multiples of NC; columns below j0 + jb (the block itself) or
// at/after ld are masked out.
__global__ void __launch_bounds__(256) k_update(LuArgs a, int j0, int jb, int strip0) {
  const int mat = blockIdx.y;
  const int cs = strip0 + blockIdx.x * NC;  // first column of the strip (multiple of NC)
  const int live0 = j0 + jb;
  double* W = a.W + (size_t)mat * a.mat_stride;
  const int* ipiv = a.ipiv + (size_t)mat * a.ipiv_stride;
  const int ld = a.ld, tid = threadIdx.x;
  __shared__ double sL[NB * NB];   // unit lower L11
  __shared__ double sU[NB * NC];   // U12 strip
  __shared__ double sP[4][NC];
  // row swaps of the block applied to the strip (sequential order)
  for (int r = 0; r < jb; ++r) {
    const int pr = ipiv[j0 + r];
    if (pr != j0 + r && tid < NC && cs + tid >= live0 && cs + tid < ld) {
      double t = W[(size_t)(j0 + r) * ld + cs + tid];
      W[(size_t)(j0 + r) * ld + cs + tid] = W[(size_t)pr * ld + cs + tid];
      W[(size_t)pr * ld + cs + tid] = t;
    }
    __syncthreads();
  }
  for (int i = tid; i < NB * NB; i += 256) {
    const int r = i / NB, c = i % NB;
    sL[i] = (r < jb && c < jb) ? W[(size_t)(j0 + r) * ld + j0 + c] : 0.0;
  }
  for (int i = tid; i < NB * NC; i += 256) {
    const int r = i / NC, c = i % NC;
    sU[i] = (r < jb && cs + c >= live0 && cs + c < ld) ? W[(size_t)(j0 + r) * ld + cs + c] : 0.0;
  }
  __syncthreads();
  // U12 = L11^{-1} A12: row by row, the sum over m split in 4 parts
  {
    const int col = tid % NC, part = tid / NC;
    for (int i = 1; i < jb; ++i) {
      double s = 0.0;
      for (int m = part; m < i; m += 4) s += sL[i * NB + m] * sU[m * NC + col];
      sP[part][col] = s;
      __syncthreads();
      if (part == 0) sU[i * NC + col] -= sP[0][col] + sP[1][col] + sP[2][col] + sP[3][col];
      __syncthreads();
    }
  }
  for (int i = tid; i < jb * NC; i += 256) {
    const int r = i / NC, c = i % NC;
    if (cs + c >= live0 && cs + c < ld) W[(size_t)(j0 + r) * ld + cs + c] = sU[i];
  }
  // A22 -= L21 U12 with FP64 MFMA: each wave takes 16-row tiles of the strip
  const int lane = tid & 63, wave = tid >> 6;
  const int row_lo = j0 + jb;
  const int ntile = (a.n_rows - row_lo + 15) / 16;
  const int kq = (jb + 3) / 4;  // k-steps of 4
  for (int tile = wave; tile < ntile; tile += 4) {
    const int r0 = row_lo + tile * 16;
    dbl4 acc[NC / 16];
#pragma unroll
    for (int ct = 0; ct < NC / 16; ++ct) {
      const int cc = cs + ct * 16 + (lane & 15);
      const bool cok = cc >= live0 && cc < ld;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = r0 + 4 * i + (lane >> 4);  // f64 16x16x4: D[4 reg + lane/16][lane%16]
        acc[ct][i] = (r < a.n_rows && cok) ? W[(size_t)r * ld + cc] : 0.0;
      }
    }
    const int ra = r0 + (lane & 15);
    for (int ks = 0; ks < kq; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      const double av = (ra < a.n_rows && kk < jb) ? -W[(size_t)ra * ld + j0 + kk] : 0.0;
#pragma unroll
      for (int ct = 0; ct < NC / 16; ++ct) {
        const double bv = (kk < jb) ? sU[kk * NC + ct * 16 + (lane & 15)] : 0.0;
        acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ct = 0; ct < NC / 16; ++ct) {
      const int cc = cs + ct * 16 + (lane & 15);
      const bool cok = cc >= live0 && cc < ld;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = r0 + 4 * i + (lane >> 4);  // f64 16x16x4: D[4 reg + lane/16][lane%16]
        if (r < a.n_rows && cok) W[(size_t)r * ld + cc] = acc[ct][i];
      }
    }
  }
}

}  // namespace

// Eliminate the first n_piv columns of `batch` matrices (see file comment).
hipError_t lu_eliminate(hipStream_t s, double* W, int batch, long long mat_stride, int ld, int n_piv, int n_rows,
                        int n_cols, int* ipiv, int ipiv_stride, int* status) {
  LuArgs a{W, mat_stride, ld, n_piv, n_rows, n_cols, ipiv, ipiv_stride, status};
  if (ld % NC != 0) return hipErrorInvalidValue;
  const int rpt = (n_piv + PANEL_THREADS - 1) / PANEL_THREADS;
  for (int j0 = 0; j0 < n_piv; j0 += NB) {
    const int jb = std::min(NB, n_piv - j0);
    if (rpt <= 1) hipLaunchKernelGGL(k_panel<1>, dim3(batch), dim3(PANEL_THREADS), 0, s, a, j0, jb);
    else if (rpt <= 2) hipLaunchKernelGGL(k_panel<2>, dim3(batch), dim3(PANEL_THREADS), 0, s, a, j0, jb);
    else if (rpt <= 4) hipLaunchKernelGGL(k_panel<4>, dim3(batch), dim3(PANEL_THREADS), 0, s, a, j0, jb);
    else if (rpt <= 8) hipLaunchKernelGGL(k_panel<8>, dim3(batch), dim3(PANEL_THREADS), 0, s, a, j0, jb);
    else return hipErrorInvalidValue;
    if (n_rows > n_piv)
      hipLaunchKernelGGL(k_dtrsm, dim3((n_rows - n_piv + 255) / 256, batch), dim3(256), 0, s, a, j0, jb);
    // strips aligned to NC covering the live columns [j0 + jb, n_cols)
    const int live0 = j0 + jb;
    const int strip0 = live0 / NC * NC;
    const int nstrip = (n_cols > live0) ? (n_cols - strip0 + NC - 1) / NC : 0;
    if (nstrip > 0) hipLaunchKernelGGL(k_update, dim3(nstrip, batch), dim3(256), 0, s, a, j0, jb, strip0);
  }
  return hipGetLastError();
}

hipError_t launch_lu(HdgContext& c) {
  return lu_eliminate(c.stream, c.ws.Wm, c.hm.n_macros, (long long)c.n_rows * c.ldw, c.ldw, c.hc.n_u, c.n_rows,
                      c.n_cols, c.ws.ipiv, c.hc.n_u, reinterpret_cast<int*>(c.ws.small));
}

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
// Columns are eliminated in pairs of NB = 64-column blocks (look-ahead):
//   k_panel   one workgroup per matrix factors the S rows of a block in
//             sub-panels of PW columns held in registers (pivot search by a
//             workgroup arg-max, first maximum wins as in LAPACK) and records
//             the block's net row permutation;
//   k_uinv + k_gemm   L of the non-pivot rows: A_D,block U11^{-1};
//   k_u12     row swaps and U12 = L11^{-1} A12 of one block for one strip
//             (used to bring the second block of a pair up to date);
//   k_linv2 + k_u12lin   the inverse of the pair's 128 x 128 unit-lower
//             diagonal block, then per 64-column strip the row swaps of both
//             blocks and U12 = L^{-1} A12 as an MFMA product;
//   k_gemm    A22 -= L21 U12 for all strips, K = 128, on MFMA
//             (v_mfma_f64_16x16x4f64 in FP64, v_mfma_f32_16x16x4f32 in FP32).
// Every kernel is a template on the storage and arithmetic type T (double or
// float); the FP32 instance is the low-precision condensation.
#include "context.h"
#include <algorithm>
#include <type_traits>

namespace {

// 16x16x4 MFMA per element type.  Operands: lane l supplies A[l % 16][k] and
// B[k][l % 16] with k = l / 16; result register i of lane l holds
// D[row(i, l / 16)][l % 16].
template <class T> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int i, int grp) { return 4 * i + grp; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int i, int grp) { return 4 * grp + i; }
};

// BF16 operands with FP32 accumulation (16x16x16): lane l supplies
// A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j][l % 16], j = 0..3; the
// result registers are laid out as for the FP32 16x16x4 instruction.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ short to_bf16(float x) {  // round to nearest even
  const unsigned u = __float_as_uint(x);
  return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

constexpr int NB = 64;     // block width of the trailing update
constexpr int PW = 16;     // sub-panel width held in registers
constexpr int PANEL_THREADS = 512;
constexpr int NC = 64;     // strip width of the trailing update

template <class T>
struct LuArgs {
  T* W;
  long long mat_stride;  // elements between matrices
  int ld, n_piv, n_rows, n_cols;
  int* ipiv;             // [batch][n_piv]
  int ipiv_stride;
  int* status;           // first singular matrix index + 1 (0 = none)
  int* perm;             // [batch][PERM_STRIDE]: net row permutation of the current block
};

// Net effect of a block's row swaps: position j0 + i takes the old row
// perm[i] (i < jb); nout further positions perm[NB + k] take perm[2 NB + k];
// perm[3 NB] = nout.
constexpr int PERM_STRIDE = 3 * 64 + 4;
// two slots per matrix (consecutive 64-column blocks alternate)
template <class T>
__device__ __forceinline__ int* perm_slot(const LuArgs<T>& a, int mat, int j0) {
  return a.perm + ((size_t)mat * 2 + ((j0 / 64) & 1)) * PERM_STRIDE;
}

template <class T>
__device__ __forceinline__ void argmax_update(T& bv, int& bi, T v, int i) {
  if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
}

template <class T, int RPT, int NT, int PWT = PW>
__global__ void __launch_bounds__(NT) k_panel(LuArgs<T> a, int j0, int jb, int lcol0) {
  const int tid = threadIdx.x;
  const int mat = blockIdx.x;
  T* W = a.W + (size_t)mat * a.mat_stride;
  int* ipiv = a.ipiv + (size_t)mat * a.ipiv_stride;
  const int ld = a.ld, n_piv = a.n_piv;
  __shared__ T s_bv[NT / 64];
  __shared__ int s_bi[NT / 64];
  __shared__ int s_prow;
  __shared__ T s_urow[PWT];
  __shared__ T s_swap[2][PWT];
  __shared__ T s_U[PWT * NB];
  __shared__ T s_L[PWT * PWT];     // unit-lower L of the sub-panel's own rows
  __shared__ int s_piv[PWT];       // pivot rows of the sub-panel's columns
  __shared__ int s_mv[2][2 * PWT];  // net row moves of the sub-panel: dst, src
  __shared__ int s_nmv;
  __shared__ T s_mvbuf[2 * PWT * 2 * NB];  // old values of the moved rows
  for (int c0 = j0; c0 < j0 + jb; c0 += PWT) {
    const int pw = min(PWT, j0 + jb - c0);
    // rows owned by this thread: c0 + tid + i * NT
    T v[RPT][PWT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = c0 + tid + i * NT;
#pragma unroll
      for (int cc = 0; cc < PWT; ++cc) v[i][cc] = (r < n_piv && cc < pw) ? W[wtix(r, c0 + cc, ld)] : T(0);
    }
    // columns of the sub-panel unrolled: register indices known at compile time
#pragma unroll
    for (int cc = 0; cc < PWT; ++cc) {
      if (cc < pw) {  // uniform
      const int col = c0 + cc;
      // pivot search over rows [col, n_piv)
      T bv = T(-1);
      int bi = 0x7fffffff;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + i * NT;
        T vc = v[i][0];
#pragma unroll
        for (int k = 1; k < PWT; ++k) vc = (k == cc) ? v[i][k] : vc;
        if (r >= col && r < n_piv) argmax_update<T>(bv, bi, fabs(vc), r);
      }
      for (int off = 32; off > 0; off >>= 1) {
        T ov = __shfl_xor(bv, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        argmax_update<T>(bv, bi, ov, oi);
      }
      if ((tid & 63) == 0) { s_bv[tid >> 6] = bv; s_bi[tid >> 6] = bi; }
      __syncthreads();
      if (tid == 0) {
        T b = s_bv[0];
        int bi0 = s_bi[0];
        for (int w = 1; w < NT / 64; ++w) argmax_update<T>(b, bi0, s_bv[w], s_bi[w]);
        if (!(b > T(0))) {  // zero or NaN column: singular
          if (a.status) atomicCAS(a.status, 0, mat + 1);
          bi0 = col;
        }
        s_prow = bi0;
        s_piv[cc] = bi0;  // to ipiv after the sub-panel (no global store before the barriers)
      }
      __syncthreads();
      const int prow = s_prow;
      // exchange rows col and prow inside the sub-panel registers
      const int oc = col - c0, op = prow - c0;
      if (prow != col) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int rl = tid + i * NT;
          if (rl == oc) {
#pragma unroll
            for (int k = 0; k < PWT; ++k) s_swap[0][k] = v[i][k];
          }
          if (rl == op) {
#pragma unroll
            for (int k = 0; k < PWT; ++k) s_swap[1][k] = v[i][k];
          }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int rl = tid + i * NT;
          if (rl == oc) {
#pragma unroll
            for (int k = 0; k < PWT; ++k) v[i][k] = s_swap[1][k];
          }
          if (rl == op) {
#pragma unroll
            for (int k = 0; k < PWT; ++k) v[i][k] = s_swap[0][k];
          }
        }
      }
      // broadcast the pivot row
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (tid + i * NT == oc) {
#pragma unroll
          for (int k = 0; k < PWT; ++k) s_urow[k] = v[i][k];
        }
      }
      __syncthreads();
      const T piv = s_urow[cc];
      const T ipv = (piv != T(0)) ? T(1) / piv : T(0);
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + i * NT;
        if (r > col && r < n_piv) {
          T vc = v[i][0];
#pragma unroll
          for (int k = 1; k < PWT; ++k) vc = (k == cc) ? v[i][k] : vc;
          const T l = vc * ipv;
#pragma unroll
          for (int k = 0; k < PWT; ++k) {
            if (k == cc) v[i][k] = l;
            if (k > cc) v[i][k] -= l * s_urow[k];
          }
        }
      }
      __syncthreads();
      }
    }
    // The sub-panel's row swaps on the rest of the block row (columns
    // [lcol0, c0) and [c0 + pw, j0 + jb); lcol0 < j0 takes the L columns of
    // the previous block too) as one net permutation: position dst takes the
    // old row src, all old values loaded before any is stored.
    if (tid == 0) {
      int* pos = s_mv[0];   // position pos[t] now holds the old row cont[t]
      int* cont = s_mv[1];
      int n = pw;
      for (int i = 0; i < pw; ++i) pos[i] = cont[i] = c0 + i;
      for (int cc = 0; cc < pw; ++cc) {
        const int pb = s_piv[cc];
        if (pb == c0 + cc) continue;
        int jb2 = -1;
        for (int t = 0; t < n; ++t)
          if (pos[t] == pb) jb2 = t;
        if (jb2 < 0) { pos[n] = cont[n] = pb; jb2 = n++; }
        const int t = cont[cc];
        cont[cc] = cont[jb2];
        cont[jb2] = t;
      }
      int m = 0;  // keep the moves (in place: m <= t)
      for (int t = 0; t < n; ++t)
        if (pos[t] != cont[t]) { pos[m] = pos[t]; cont[m] = cont[t]; ++m; }
      s_nmv = m;
    }
    __syncthreads();
    if (tid < pw) ipiv[c0 + tid] = s_piv[tid];
    const int nmv = s_nmv, nbr = j0 + jb - lcol0;  // nbr <= 2 NB columns
    if (nmv > 0) {
      for (int x = tid; x < nmv * nbr; x += NT) {
        const int t = x / nbr, cidx = lcol0 + x % nbr;
        if (cidx < c0 || cidx >= c0 + pw) s_mvbuf[x] = W[wtix(s_mv[1][t], cidx, ld)];
      }
      __syncthreads();
      for (int x = tid; x < nmv * nbr; x += NT) {
        const int t = x / nbr, cidx = lcol0 + x % nbr;
        if (cidx < c0 || cidx >= c0 + pw) W[wtix(s_mv[0][t], cidx, ld)] = s_mvbuf[x];
      }
    }
    // write the factored sub-panel back; its own L rows also to LDS
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = c0 + tid + i * NT;
      if (r < n_piv) {
#pragma unroll
        for (int cc = 0; cc < PWT; ++cc)
          if (cc < pw) W[wtix(r, c0 + cc, ld)] = v[i][cc];
      }
    }
    if (tid < pw) {
#pragma unroll
      for (int cc = 0; cc < PWT; ++cc) s_L[tid * PWT + cc] = v[0][cc];
    }
    // right-looking update of the rest of the block: columns [c0 + pw, j0 + jb)
    const int rest0 = c0 + pw, nrest = j0 + jb - rest0;
    __syncthreads();
    if (nrest > 0) {
      // U rows of the sub-panel: L_sub^{-1} A[c0:c0+pw, rest]  (unit lower, sequential rows)
      for (int k = tid; k < nrest; k += NT) {
#pragma unroll 4
        for (int i = 0; i < pw; ++i) s_U[i * NB + k] = W[wtix((c0 + i), rest0 + k, ld)];
        for (int i = 1; i < pw; ++i) {
          T s = s_U[i * NB + k];
          for (int m = 0; m < i; ++m) s -= s_L[i * PWT + m] * s_U[m * NB + k];
          s_U[i * NB + k] = s;
        }
      }
      __syncthreads();
      for (int k = tid; k < pw * nrest; k += NT) {
        const int i = k / nrest, cidx = k % nrest;
        W[wtix((c0 + i), rest0 + cidx, ld)] = s_U[i * NB + cidx];
      }
      // rows below the sub-panel: A[r, rest] -= L[r, c0:c0+pw] U, CB
      // columns of all the thread's rows loaded at once (16 loads in flight
      // per thread); with many rows per thread (register budget) row by row
      constexpr int CB = RPT >= 16 ? 1 : 16 / RPT;
      if constexpr (RPT >= 16) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int r = c0 + tid + i * NT;
          if (r >= c0 + pw && r < n_piv) {
#pragma unroll 4
            for (int cidx = 0; cidx < nrest; ++cidx) {
              T s = W[wtix(r, rest0 + cidx, ld)];
#pragma unroll
              for (int m = 0; m < PWT; ++m)
                if (m < pw) s -= v[i][m] * s_U[m * NB + cidx];
              W[wtix(r, rest0 + cidx, ld)] = s;
            }
          }
        }
      } else
      for (int cb = 0; cb < nrest; cb += CB) {
        T x[RPT][CB];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int r = c0 + tid + i * NT;
#pragma unroll
          for (int q = 0; q < CB; ++q)
            x[i][q] = (r >= c0 + pw && r < n_piv && cb + q < nrest) ? W[wtix(r, rest0 + cb + q, ld)] : T(0);
        }
#pragma unroll
        for (int q = 0; q < CB; ++q) {
          if (cb + q >= nrest) break;
#pragma unroll
          for (int m = 0; m < PWT; ++m) {
            if (m < pw) {
              const T um = s_U[m * NB + cb + q];
#pragma unroll
              for (int i = 0; i < RPT; ++i) x[i][q] -= v[i][m] * um;
            }
          }
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int r = c0 + tid + i * NT;
#pragma unroll
          for (int q = 0; q < CB; ++q)
            if (r >= c0 + pw && r < n_piv && cb + q < nrest) W[wtix(r, rest0 + cb + q, ld)] = x[i][q];
        }
      }
      __syncthreads();
    }
  }
  // net row permutation of the block's swaps, for the strips to the right
  if (tid == 0) {
    int* pm = perm_slot(a, mat, j0);
    int s_in[NB];
    int nout = 0;
    for (int i = 0; i < NB; ++i) s_in[i] = j0 + i;
    for (int r = 0; r < jb; ++r) {
      const int pa = j0 + r, pb = ipiv[pa];
      if (pb == pa) continue;
      int* src_b = nullptr;
      if (pb < j0 + jb) {
        src_b = &s_in[pb - j0];
      } else {
        for (int k = 0; k < nout; ++k)
          if (pm[NB + k] == pb) { src_b = &pm[2 * NB + k]; break; }
        if (!src_b) { pm[NB + nout] = pb; pm[2 * NB + nout] = pb; src_b = &pm[2 * NB + nout]; ++nout; }
      }
      const int t = s_in[r];
      s_in[r] = *src_b;
      *src_b = t;
    }
    for (int i = 0; i < NB; ++i) pm[i] = s_in[i];
    pm[3 * NB] = nout;
  }
}

// ---- tournament pivoting of one block ------------------------------------
// Communication-avoiding choice of the block's pivot rows: every workgroup
// factors up to TR rows of the block with partial pivoting (rows stay with
// their thread, the chosen ones are marked) and hands on the rows it chose;
// the chosen rows of up to TSETS groups meet again in the next round until
// one group is left.  That group's pivot order is the block's row order; its
// rows, factored once more in that order (no pivoting: the same arithmetic),
// give L11 \ U11.  The last round also moves the rows (the block, and the L
// columns from lcol0 of the previous block) and records ipiv and the net
// permutation as k_panel does.  The rows below the block then get
// L21 = A21 U11^{-1} from k_uinv + k_gemm, as the non-pivot rows always do.
constexpr int TR = 256;                 // rows per tournament group (one per thread)
constexpr int TSETS = TR / NB;          // candidate sets that meet in one group
constexpr int TMAXG = 12 * 1024 / TR;   // first-round groups for up to 12288 pivot rows
constexpr int TMOVE = 48;               // moved values per thread in the last round

template <class T>
__device__ __forceinline__ T piv_mag(T x) {  // |x| with NaN read as 0 (a row is always chosen)
  const T m = fabs(x);
  return (m >= T(0)) ? m : T(0);
}

// The block's columns of the thread's row in v[0 .. NB) (window shifted by 8
// columns per sub-panel); steps of partial pivoting over the rows with
// active = true.  chosen[j] receives the row picked at step j (or -1), the
// picked rows turn inactive.  With `track`, *bmin receives the smallest pivot
// magnitude (for the singularity flag).
template <class T>
__device__ __forceinline__ void tslu_steps(T (&v)[NB], int row, bool& active, int jb, T* s_bv, int* s_bi, T* s_urow,
                                           int* chosen, T* bmin) {
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < jb; c0 += 8) {
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      if (c0 + cc < jb) {  // uniform
        T bv = active ? piv_mag<T>(v[cc]) : T(-1);
        int bi = active ? row : 0x7fffffff;
        for (int off = 32; off > 0; off >>= 1) {
          const T ov = __shfl_xor(bv, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          argmax_update<T>(bv, bi, ov, oi);
        }
        if ((tid & 63) == 0) { s_bv[tid >> 6] = bv; s_bi[tid >> 6] = bi; }
        __syncthreads();
        T b = s_bv[0];
        int w = s_bi[0];
#pragma unroll
        for (int q = 1; q < TR / 64; ++q) argmax_update<T>(b, w, s_bv[q], s_bi[q]);
        const bool mine = active && row == w;
        if (mine) {
          active = false;
#pragma unroll
          for (int k = 0; k < NB; ++k) s_urow[k] = v[k];
        }
        if (tid == 0) {
          chosen[c0 + cc] = (b >= T(0)) ? w : -1;
          if (bmin && b < *bmin) *bmin = b;
        }
        __syncthreads();
        if (active) {
          const T piv = s_urow[cc];
          const T ipv = (piv != T(0)) ? T(1) / piv : T(0);
          const T l = v[cc] * ipv;
          v[cc] = l;
#pragma unroll
          for (int k = cc + 1; k < NB; ++k) v[k] -= l * s_urow[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NB - 8; ++k) v[k] = v[k + 8];
#pragma unroll
    for (int k = NB - 8; k < NB; ++k) v[k] = T(0);
  }
}

// One round of the tournament: group g of matrix blockIdx.y takes the rows
// [j0 + g TR, j0 + (g + 1) TR) below n_piv (cand_in == null) or the candidate
// sets [g TSETS, (g + 1) TSETS) of cand_in (n_in sets, -1 = no row) and
// writes the rows it chose to set g of cand_out.
template <class T>
__global__ void __launch_bounds__(TR) k_tslu_round(LuArgs<T> a, int j0, int jb, const int* __restrict__ cand_in,
                                                   int n_in, int* __restrict__ cand_out) {
  const int tid = threadIdx.x, g = blockIdx.x, mat = blockIdx.y;
  const T* W = a.W + (size_t)mat * a.mat_stride;
  const int ld = a.ld;
  __shared__ T s_bv[TR / 64];
  __shared__ int s_bi[TR / 64];
  __shared__ T s_urow[NB];
  __shared__ int s_win[NB];
  int row;
  if (cand_in == nullptr) {
    row = j0 + g * TR + tid;
    if (row >= a.n_piv) row = -1;
  } else {
    const int set = g * TSETS + tid / NB, i = tid % NB;
    row = (set < n_in && i < jb) ? cand_in[((size_t)mat * TMAXG + set) * NB + i] : -1;
  }
  T v[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) v[k] = (row >= 0 && k < jb) ? W[wtix(row, j0 + k, ld)] : T(0);
  bool active = row >= 0;
  tslu_steps<T>(v, row, active, jb, s_bv, s_bi, s_urow, s_win, nullptr);
  if (tid < NB) cand_out[((size_t)mat * TMAXG + g) * NB + tid] = tid < jb ? s_win[tid] : -1;
}

// Last round (one group per matrix): the pivot order, L11 \ U11 of the chosen
// rows, the row moves, ipiv (LAPACK sequential-swap form) and the net
// permutation of the block.
template <class T>
__global__ void __launch_bounds__(TR) k_tslu_final(LuArgs<T> a, int j0, int jb, int lcol0,
                                                   const int* __restrict__ cand_in, int n_in) {
  const int tid = threadIdx.x, mat = blockIdx.x;
  T* W = a.W + (size_t)mat * a.mat_stride;
  int* ipiv = a.ipiv + (size_t)mat * a.ipiv_stride;
  const int ld = a.ld;
  __shared__ T s_bv[TR / 64];
  __shared__ int s_bi[TR / 64];
  __shared__ T s_urow[NB];
  __shared__ int s_win[NB];
  __shared__ T s_bmin;
  __shared__ T s_top[NB * NB];        // L11 \ U11, row j = the row chosen at step j
  __shared__ int s_pos[2 * NB], s_cont[2 * NB];
  __shared__ int s_n;
  int row;
  if (cand_in == nullptr) {
    row = j0 + tid;
    if (row >= a.n_piv || tid >= TR) row = -1;
  } else {
    const int set = tid / NB, i = tid % NB;
    row = (set < n_in && i < jb) ? cand_in[((size_t)mat * TMAXG + set) * NB + i] : -1;
  }
  if (tid == 0) s_bmin = T(1);
  T v[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) v[k] = (row >= 0 && k < jb) ? W[wtix(row, j0 + k, ld)] : T(0);
  bool active = row >= 0;
  __syncthreads();
  tslu_steps<T>(v, row, active, jb, s_bv, s_bi, s_urow, s_win, &s_bmin);
  if (tid == 0 && !(s_bmin > T(0)) && a.status) atomicCAS(a.status, 0, mat + 1);
  // the chosen rows again, in pivot order, without pivoting: row j on thread j
  const int prow = tid < jb ? s_win[tid] : -1;
#pragma unroll
  for (int k = 0; k < NB; ++k) v[k] = (prow >= 0 && k < jb) ? W[wtix(prow, j0 + k, ld)] : T(0);
  for (int c0 = 0; c0 < jb; c0 += 8) {
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int j = c0 + cc;
      if (j < jb) {
        if (tid == j) {
#pragma unroll
          for (int k = 0; k < NB; ++k) s_urow[k] = v[k];
        }
        __syncthreads();
        if (tid > j && tid < jb) {
          const T piv = s_urow[cc];
          const T ipv = (piv != T(0)) ? T(1) / piv : T(0);
          const T l = v[cc] * ipv;
          v[cc] = l;
#pragma unroll
          for (int k = cc + 1; k < NB; ++k) v[k] -= l * s_urow[k];
        }
        __syncthreads();
      }
    }
    if (tid < jb) {
#pragma unroll
      for (int cc = 0; cc < 8; ++cc)
        if (c0 + cc < jb) s_top[tid * NB + c0 + cc] = v[cc];
    }
#pragma unroll
    for (int k = 0; k < NB - 8; ++k) v[k] = v[k + 8];
#pragma unroll
    for (int k = NB - 8; k < NB; ++k) v[k] = T(0);
  }
  // sequential swaps: position j0 + j takes the row chosen at step j from
  // where it is now (wave 0 searches the touched positions in parallel)
  if (tid < 64) {
    for (int i = tid; i < 2 * NB; i += 64) { s_pos[i] = j0 + i; s_cont[i] = j0 + i; }
    int n = jb;
    for (int j = 0; j < jb; ++j) {
      const int pb = s_win[j];
      int t = -1;
      for (int i = tid; i < n; i += 64)
        if (s_cont[i] == pb) t = i;
      // at most one lane holds the row
      for (int off = 32; off > 0; off >>= 1) t = max(t, __shfl_xor(t, off, 64));
      if (t < 0) {  // untouched row below the block: add its position
        t = n;
        if (tid == 0) { s_pos[n] = pb; s_cont[n] = pb; }
        ++n;
      }
      if (tid == 0) {
        ipiv[j0 + j] = s_pos[t];
        const int x = s_cont[j];
        s_cont[j] = s_cont[t];
        s_cont[t] = x;
      }
      // lane 0's LDS writes reach the wave before the next search
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    if (tid == 0) s_n = n;
  }
  __syncthreads();
  const int n = s_n;
  // net permutation for the strips to the right (k_u12, k_u12lin)
  if (tid == 0) {
    int* pm = perm_slot(a, mat, j0);
    int nout = 0;
    for (int i = 0; i < NB; ++i) pm[i] = i < jb ? s_cont[i] : j0 + i;
    for (int t = jb; t < n; ++t)
      if (s_pos[t] != s_cont[t]) { pm[NB + nout] = s_pos[t]; pm[2 * NB + nout] = s_cont[t]; ++nout; }
    pm[3 * NB] = nout;
  }
  // row moves in columns [lcol0, j0 + jb): positions j0 .. j0 + jb - 1 take the
  // chosen rows (columns left of the block moved, block columns from s_top),
  // positions t >= jb of the list take the rows displaced from the top (all
  // columns); every old value is read before any is written
  const int nl = j0 - lcol0, nw = j0 + jb - lcol0;
  const int n_top = jb * nl, n_all = n_top + (n - jb) * nw;
  T buf[TMOVE];
#pragma unroll
  for (int i = 0; i < TMOVE; ++i) {
    const int x = tid + i * TR;
    buf[i] = T(0);
    if (x < n_top) {
      const int m = x / nl, col = lcol0 + x % nl;
      if (s_cont[m] != j0 + m) buf[i] = W[wtix(s_cont[m], col, ld)];
    } else if (x < n_all) {
      const int y = x - n_top, t = jb + y / nw, col = lcol0 + y % nw;
      if (s_pos[t] != s_cont[t]) buf[i] = W[wtix(s_cont[t], col, ld)];
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // every load has returned before any store below
  __syncthreads();
#pragma unroll
  for (int i = 0; i < TMOVE; ++i) {
    const int x = tid + i * TR;
    if (x < n_top) {
      const int m = x / nl, col = lcol0 + x % nl;
      if (s_cont[m] != j0 + m) W[wtix(j0 + m, col, ld)] = buf[i];
    } else if (x < n_all) {
      const int y = x - n_top, t = jb + y / nw, col = lcol0 + y % nw;
      if (s_pos[t] != s_cont[t]) W[wtix(s_pos[t], col, ld)] = buf[i];
    }
  }
  for (int x = tid; x < jb * jb; x += TR) {
    const int r = x / jb, col = x % jb;
    W[wtix(j0 + r, j0 + col, ld)] = s_top[r * NB + col];
  }
}

// U11^{-1} of the block (identity-padded to NB x NB) into Uinv[mat]: one
// thread per column, backward substitution in LDS.
template <class T>
__global__ void __launch_bounds__(64) k_uinv(LuArgs<T> a, int j0, int jb, T* __restrict__ Uinv) {
  const int mat = blockIdx.x;
  const T* W = a.W + (size_t)mat * a.mat_stride;
  const int ld = a.ld;
  __shared__ T sU[NB * NB];
  __shared__ T sI[NB * NB];
  for (int i = threadIdx.x; i < NB * NB; i += blockDim.x) {
    const int r = i / NB, c = i % NB;
    T v = (r == c) ? T(1) : T(0);
    if (r < jb && c < jb) v = W[wtix((j0 + r), j0 + c, ld)];
    sU[i] = v;
  }
  __syncthreads();
  const int j = threadIdx.x;
  for (int i = NB - 1; i >= 0; --i) {
    T s = (i == j) ? T(1) : T(0);
    for (int m = i + 1; m <= j; ++m) s -= sU[i * NB + m] * sI[m * NB + j];
    const T dgl = sU[i * NB + i];
    sI[i * NB + j] = (i <= j && dgl != T(0)) ? s / dgl : T(0);
  }
  __syncthreads();
  T* out = Uinv + (size_t)mat * NB * NB;
  for (int i = threadIdx.x; i < NB * NB; i += blockDim.x) out[i] = sI[i];
}

// Row swaps of the block and U12 = L11^{-1} A12 for one 64-column strip,
// written back in place (rows [j0, j0 + jb) of the strip).  Columns below
// live0 = j0 + jb or at/after ld are left alone.
template <class T>
__global__ void __launch_bounds__(256) k_u12(LuArgs<T> a, int j0, int jb, int strip0, int col_end) {
  const int mat = blockIdx.y;
  const int cs = strip0 + blockIdx.x * NC;
  const int live0 = j0 + jb;
  T* W = a.W + (size_t)mat * a.mat_stride;
  const int* pm = perm_slot(a, mat, j0);
  const int ld = a.ld, tid = threadIdx.x;
  __shared__ T sL[NB * NB];
  __shared__ T sU[NB * NC];
  __shared__ T sP[4][NC];
  __shared__ int s_src[2 * NB], s_dst[2 * NB];
  // the block's swaps as one gather: block rows and the nout rows outside it
  const int nout = pm[3 * NB];
  for (int i = tid; i < jb; i += 256) { s_dst[i] = j0 + i; s_src[i] = pm[i]; }
  for (int k = tid; k < nout; k += 256) { s_dst[jb + k] = pm[NB + k]; s_src[jb + k] = pm[2 * NB + k]; }
  __syncthreads();
  const int nt = jb + nout;
  const int c = tid & (NC - 1);
  const bool cok = cs + c >= live0 && cs + c < col_end;
  // each thread gathers the values of its column for touched rows p = tid/64 + 4 j
  T gv[2 * NB / 4];
#pragma unroll
  for (int j = 0; j < 2 * NB / 4; ++j) {
    const int p = (tid >> 6) + 4 * j;
    gv[j] = (p < nt && cok) ? W[wtix(s_src[p], cs + c, ld)] : T(0);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 2 * NB / 4; ++j) {
    const int p = (tid >> 6) + 4 * j;
    if (p < nt && cok) {
      if (p >= jb) W[wtix(s_dst[p], cs + c, ld)] = gv[j];  // rows outside the block
      else sU[p * NC + c] = gv[j];                             // block rows: to LDS for the solve
    }
  }
  for (int i = tid; i < NB * NB; i += 256) {
    const int r = i / NB, cc = i % NB;
    sL[i] = (r < jb && cc < jb) ? W[wtix((j0 + r), j0 + cc, ld)] : T(0);
  }
  for (int i = tid; i < NB * NC; i += 256) {
    const int r = i / NC, cc = i % NC;
    if (!(r < jb && cs + cc >= live0 && cs + cc < col_end)) sU[i] = T(0);
  }
  __syncthreads();
  {
    const int col = tid % NC, part = tid / NC;
    for (int i = 1; i < jb; ++i) {
      T s = T(0);
      for (int m = part; m < i; m += 4) s += sL[i * NB + m] * sU[m * NC + col];
      sP[part][col] = s;
      __syncthreads();
      if (part == 0) sU[i * NC + col] -= sP[0][col] + sP[1][col] + sP[2][col] + sP[3][col];
      __syncthreads();
    }
  }
  for (int i = tid; i < jb * NC; i += 256) {
    const int r = i / NC, c = i % NC;
    if (cs + c >= live0 && cs + c < col_end) W[wtix((j0 + r), cs + c, ld)] = sU[i];
  }
}

// Inverse of the unit-lower 128 x 128 diagonal block of two consecutive
// 64-column blocks b1 = [j0, j0 + 64), b2 = [j0 + 64, j0 + 64 + jb2):
//   L = [[L11, 0], [L21, L22]],  L^{-1} = [[L11^{-1}, 0], [-L22^{-1} L21 L11^{-1}, L22^{-1}]],
// identity-padded beyond 64 + jb2, row-major into Linv[mat] (128 x 128).
// One workgroup per matrix, two 64 x 64 LDS buffers (66.5 KB, so that it
// fits on a CU beside one trailing-update workgroup): L11^{-1} by forward
// substitution, X = L21 L11^{-1}, then -L22^{-1} X and L22^{-1} by forward
// substitution with L22, one column per thread.
template <class T>
__global__ void __launch_bounds__(256) k_linv2(LuArgs<T> a, int j0, int jb2, T* __restrict__ Linv) {
  const int mat = blockIdx.x, tid = threadIdx.x;
  const T* W = a.W + (size_t)mat * a.mat_stride;
  const int ld = a.ld;
  __shared__ T sA[NB][NB + 1];
  __shared__ T sB[NB][NB + 1];
  T* out = Linv + (size_t)mat * 4 * NB * NB;
  // sA <- strict lower part of L11
  for (int i = tid; i < NB * NB; i += 256) {
    const int r = i / NB, c = i % NB;
    sA[r][c] = (c < r) ? W[wtix(j0 + r, j0 + c, ld)] : T(0);
  }
  __syncthreads();
  if (tid < NB) {  // sB <- L11^{-1}, column tid
    const int j = tid;
    for (int i = 0; i < NB; ++i) {
      T x = (i == j) ? T(1) : T(0);
      if (i > j)
        for (int k = j; k < i; ++k) x -= sA[i][k] * sB[k][j];
      sB[i][j] = (i >= j) ? x : T(0);
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    out[(size_t)r * 2 * NB + c] = sB[r][c];
    out[(size_t)r * 2 * NB + NB + c] = T(0);
  }
  // sA <- X = L21 L11^{-1} (rows beyond jb2 are zero)
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    T s = T(0);
    if (r < jb2)
      for (int k = c; k < NB; ++k) s += W[wtix(j0 + NB + r, j0 + k, ld)] * sB[k][c];
    sA[r][c] = s;
  }
  __syncthreads();
  // sB <- strict lower part of L22 (zero beyond jb2)
  for (int i = tid; i < NB * NB; i += 256) {
    const int r = i / NB, c = i % NB;
    sB[r][c] = (c < r && r < jb2) ? W[wtix(j0 + NB + r, j0 + NB + c, ld)] : T(0);
  }
  __syncthreads();
  if (tid < NB) {  // sA <- -L22^{-1} X in place, column tid
    const int j = tid;
    for (int i = 0; i < NB; ++i) {
      T x = -sA[i][j];
      for (int k = 0; k < i; ++k) x -= sB[i][k] * sA[k][j];
      sA[i][j] = x;
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    out[(size_t)(NB + r) * 2 * NB + c] = sA[r][c];
  }
  __syncthreads();
  if (tid < NB) {  // sA <- L22^{-1}, column tid
    const int j = tid;
    for (int i = 0; i < NB; ++i) {
      T x = (i == j) ? T(1) : T(0);
      if (i > j)
        for (int k = j; k < i; ++k) x -= sB[i][k] * sA[k][j];
      sA[i][j] = (i >= j) ? x : T(0);
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    out[(size_t)(NB + r) * 2 * NB + NB + c] = sA[r][c];
  }
}

// Two consecutive 64-column blocks applied to one 64-column strip right of
// both: the row swaps of b1 then b2 (as gathers), then
//   [U12_1; U12_2] = L^{-1} [A12_1; A12_2]
// with the 128 x 128 inverse of k_linv2, on MFMA, written back to the rows
// [j0, j0 + 64 + jb2) of the strip.
template <class T>
__global__ void __launch_bounds__(256) k_u12lin(LuArgs<T> a, int j0, int jb2, int strip0, const T* __restrict__ Linv) {
  typedef typename Mfma<T>::v4 v4;
  const int mat = blockIdx.y;
  const int cs = strip0 + blockIdx.x * NC;
  const int live0 = j0 + NB + jb2;
  T* W = a.W + (size_t)mat * a.mat_stride;
  const int ld = a.ld, tid = threadIdx.x;
  __shared__ T sB[2 * NB * NC];
  __shared__ int s_src[2 * NB], s_dst[2 * NB];
  const int c = tid & (NC - 1);
  const bool cok = cs + c >= live0 && cs + c < ld;
  for (int blk = 0; blk < 2; ++blk) {
    const int jj = j0 + blk * NB, jbb = blk ? jb2 : NB;
    const int* pm = perm_slot(a, mat, jj);
    const int nout = pm[3 * NB];
    for (int i = tid; i < jbb; i += 256) { s_dst[i] = jj + i; s_src[i] = pm[i]; }
    for (int k = tid; k < nout; k += 256) { s_dst[jbb + k] = pm[NB + k]; s_src[jbb + k] = pm[2 * NB + k]; }
    __syncthreads();
    const int nt = jbb + nout;
    T gv[2 * NB / 4];
#pragma unroll
    for (int j = 0; j < 2 * NB / 4; ++j) {
      const int p = (tid >> 6) + 4 * j;
      gv[j] = (p < nt && cok) ? W[wtix(s_src[p], cs + c, ld)] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2 * NB / 4; ++j) {
      const int p = (tid >> 6) + 4 * j;
      if (p < nt && cok) W[wtix(s_dst[p], cs + c, ld)] = gv[j];
    }
    __syncthreads();
  }
  const int nr = NB + jb2;
  for (int i = tid; i < 2 * NB * NC; i += 256) {
    const int r = i / NC, cc = i % NC;
    const bool ok = r < nr && cs + cc >= live0 && cs + cc < ld;
    sB[i] = ok ? W[wtix(j0 + r, cs + cc, ld)] : T(0);
  }
  __syncthreads();
  constexpr int KS = 2 * NB / 4;  // k-steps per lane group (K = 128)
  const int lane = tid & 63, wave = tid >> 6, grp = lane >> 4, col = lane & 15;
  const T* Lm = Linv + (size_t)mat * 4 * NB * NB;
  for (int t = wave; t < 2 * NB / 16; t += 4) {
    const int r0 = t * 16;
    if (r0 >= nr) break;
    T af[KS];
    const T* ap = Lm + (size_t)(r0 + col) * 2 * NB + KS * grp;
#pragma unroll
    for (int s = 0; s < KS; ++s) af[s] = ap[s];
    v4 acc[NC / 16];
#pragma unroll
    for (int ct = 0; ct < NC / 16; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[ct][i] = T(0);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int ct = 0; ct < NC / 16; ++ct)
        acc[ct] = Mfma<T>::op(af[s], sB[(KS * grp + s) * NC + ct * 16 + col], acc[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < NC / 16; ++ct) {
      const int cc = cs + ct * 16 + col;
      if (cc < live0 || cc >= ld) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = r0 + Mfma<T>::row(i, grp);
        if (r < nr) W[wtix(j0 + r, cc, ld)] = acc[ct][i];
      }
    }
  }
}

// C[r, cs:cs+64] = (beta ? C : 0) + alpha * A[r, ak0:ak0+K] * B[0:K, 0:64] on
// FP64 MFMA for the rows [r_lo, r_hi) of one matrix, 16-row tiles, four waves
// per workgroup and `TPW` tiles per wave.  B (K x 64, leading dimension ldb)
// is staged in LDS.  The k index of an MFMA step is k = 16 (lane / 16) + step,
// so every lane loads 16 consecutive A values of its row.  Columns outside
// [c_lo, ld) are masked (read as 0, never written).
template <class T>
struct GemmArgs {
  T* W;
  long long mat_stride;
  int ld;
  const T* B;
  long long b_mat_stride;
  int ldb;
  int b_col_follow;  // 1: B = rows [b_row0, b_row0 + K) of the strip in W itself; 0: plain K x 64 B
  int b_row0;
  int ak0, K, cs0, c_lo, c_hi, r_lo, r_hi;
  T alpha;
  int beta;
  int tiles_per_wg;
  int gx, gy;        // strips and row groups per matrix (one-dimensional grid of gx gy batch workgroups)
};

// Workgroups go to the 8 XCDs round-robin (workgroup id modulo 8).  Renumber
// them so that every XCD takes one contiguous run of work items: consecutive
// items are consecutive strips of the same rows and matrix, so the rows of
// L21 they all read stay in that XCD's L2 instead of being fetched by each XCD.
__device__ __forceinline__ unsigned xcd_work_item(unsigned id, unsigned n) {
  const unsigned x = id % 8u, s = id / 8u, q = n / 8u, r = n % 8u;
  return (x < r ? x * (q + 1u) : r * (q + 1u) + (x - r) * q) + s;
}

template <class T, int KB, int NT, bool PIPE, bool B16 = false>
__device__ __forceinline__ void gemm_body(const GemmArgs<T>& g) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int KS = KB / 4;  // MFMA k-steps; lane group grp covers k in [KS grp, KS grp + KS)
  const unsigned wi = xcd_work_item(blockIdx.x, gridDim.x);
  const int strip = (int)(wi % (unsigned)g.gx), rgrp = (int)((wi / (unsigned)g.gx) % (unsigned)g.gy);
  const int mat = (int)(wi / ((unsigned)g.gx * (unsigned)g.gy));
  const int cs = g.cs0 + strip * NC;
  T* W = g.W + (size_t)mat * g.mat_stride;
  const T* B = g.B + (size_t)mat * g.b_mat_stride;
  const int ld = g.ld, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = lane >> 4, col = lane & 15;
  __shared__ T sB[KB * NC];
  for (int i = tid; i < KB * NC; i += NT) {
    const int k = i / NC, c = i % NC;
    sB[i] = (k < g.K && cs + c >= g.c_lo && cs + c < g.c_hi) ? (g.b_col_follow ? W[wtix(g.b_row0 + k, cs + c, ld)] : B[(size_t)k * g.ldb + c]) : T(0);
  }
  __syncthreads();
  const int tile0 = rgrp * g.tiles_per_wg;
  auto load_a = [&](int r0, T* af) {
    const int ra = r0 + col;
    const int kb = KS * grp;
    // the KS consecutive columns of a lane group lie inside one 64-column tile
    const T* ap = W + wtix(ra, g.ak0 + kb, ld);
    if (ra < g.r_hi && kb + KS <= g.K) {  // fast path: unmasked contiguous loads
#pragma unroll
      for (int s = 0; s < KS; ++s) af[s] = g.alpha * ap[s];
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s) af[s] = (ra < g.r_hi && kb + s < g.K) ? g.alpha * ap[s] : T(0);
    }
  };
  auto load_c = [&](int r0, v4* acc) {
#pragma unroll
    for (int ct = 0; ct < NC / 16; ++ct) {
      const int cc = cs + ct * 16 + col;
      const bool cok = cc >= g.c_lo && cc < g.c_hi;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = r0 + Mfma<T>::row(i, grp);
        acc[ct][i] = (g.beta && r < g.r_hi && cok) ? W[wtix(r, cc, ld)] : T(0);
      }
    }
  };
  auto store_c = [&](int r0, const v4* acc) {
#pragma unroll
    for (int ct = 0; ct < NC / 16; ++ct) {
      const int cc = cs + ct * 16 + col;
      const bool cok = cc >= g.c_lo && cc < g.c_hi;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = r0 + Mfma<T>::row(i, grp);
        if (r < g.r_hi && cok) W[wtix(r, cc, ld)] = acc[ct][i];
      }
    }
  };
  auto mma = [&](const T* af, v4* acc) {
    if constexpr (B16) {
      // four k values per lane and instruction: k = KS grp + 4 s4 + j
#pragma unroll
      for (int s4 = 0; s4 < KS / 4; ++s4) {
        bf16x4 a4;
#pragma unroll
        for (int j = 0; j < 4; ++j) a4[j] = to_bf16(af[4 * s4 + j]);
#pragma unroll
        for (int ct = 0; ct < NC / 16; ++ct) {
          bf16x4 b4;
#pragma unroll
          for (int j = 0; j < 4; ++j) b4[j] = to_bf16(sB[(KS * grp + 4 * s4 + j) * NC + ct * 16 + col]);
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a4, b4, acc[ct], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int ct = 0; ct < NC / 16; ++ct) {
          const T bv = sB[(KS * grp + s) * NC + ct * 16 + col];
          acc[ct] = Mfma<T>::op(af[s], bv, acc[ct]);
        }
      }
    }
  };
  T af[KS];
  v4 acc[NC / 16];
  if constexpr (PIPE) {
    // one tile with masks: C is loaded after A and added after the MFMA chain,
    // so its latency hides behind the chain (the chain starts from zero)
    auto masked_tile = [&](int r0) {
      v4 cv[NC / 16];
      load_a(r0, af);
      load_c(r0, cv);
#pragma unroll
      for (int ct = 0; ct < NC / 16; ++ct) acc[ct] = v4{T(0), T(0), T(0), T(0)};
      mma(af, acc);
#pragma unroll
      for (int ct = 0; ct < NC / 16; ++ct) acc[ct] += cv[ct];
      store_c(r0, acc);
    };
    constexpr int WST = NT / 64;  // waves per workgroup: the tile stride of a wave
    int t = wave;
    // Whole tiles of an aligned strip (rows from a multiple of 16, all 64
    // columns live, full K): A of the wave's next tile is loaded before the
    // MFMA chain of the current one; C comes from the tile's base without
    // masks at the start of the tile and joins after the chain, with alpha.
    const bool aligned = g.beta && (g.r_lo & 15) == 0 && cs >= g.c_lo && cs + NC <= g.c_hi && g.K == KB;
    if (aligned) {
      auto full = [&](int tt) { return tt < g.tiles_per_wg && g.r_lo + (tile0 + tt) * 16 + 16 <= g.r_hi; };
      auto load_a_full = [&](int r0, T* dst) {
        const T* ap = W + wtix(r0 + col, g.ak0 + KS * grp, ld);
#pragma unroll
        for (int s = 0; s < KS; ++s) dst[s] = ap[s];
      };
      T an[KS];
      if (full(t)) load_a_full(g.r_lo + (tile0 + t) * 16, an);
      for (; full(t); t += WST) {
        const int r0 = g.r_lo + (tile0 + t) * 16;
#pragma unroll
        for (int s = 0; s < KS; ++s) af[s] = an[s];
        // unconditional (the current tile again when there is no next whole
        // tile), so that the loads stay in this block ahead of the chain
        load_a_full(full(t + WST) ? r0 + 16 * WST : r0, an);
        T* cp = W + wtix(r0, cs, ld);  // the 16 x 64 tile, contiguous
        v4 cv[NC / 16];
#pragma unroll
        for (int ct = 0; ct < NC / 16; ++ct)
#pragma unroll
          for (int i = 0; i < 4; ++i) cv[ct][i] = cp[Mfma<T>::row(i, grp) * NC + ct * 16 + col];
        // keep the loads above ahead of the chain (the scheduler would sink
        // them next to their uses)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ct = 0; ct < NC / 16; ++ct) acc[ct] = v4{T(0), T(0), T(0), T(0)};
        mma(af, acc);
#pragma unroll
        for (int ct = 0; ct < NC / 16; ++ct)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            cp[Mfma<T>::row(i, grp) * NC + ct * 16 + col] = cv[ct][i] + g.alpha * acc[ct][i];
      }
    }
    // the rest (all tiles when not aligned, else a last partial tile)
    for (; t < g.tiles_per_wg; t += WST) {
      const int r0 = g.r_lo + (tile0 + t) * 16;
      if (r0 >= g.r_hi) break;
      masked_tile(r0);
    }
  } else {
    for (int t = wave; t < g.tiles_per_wg; t += NT / 64) {
      const int r0 = g.r_lo + (tile0 + t) * 16;
      if (r0 >= g.r_hi) break;
      load_a(r0, af);
      load_c(r0, acc);
      mma(af, acc);
      store_c(r0, acc);
    }
  }
}

// Four waves (256 threads); at most two workgroups per CU for FP64 (LDS).
// C joins after the MFMA chain (see gemm_body).
template <class T, int KB>
__global__ void __launch_bounds__(256, 2) k_gemm(GemmArgs<T> g) {
  gemm_body<T, KB, 256, true>(g);
}

// The trailing update with BF16 operands and FP32 accumulation (FP32 storage).
template <int KB>
__global__ void __launch_bounds__(256, 2) k_gemm_bf16(GemmArgs<float> g) {
  gemm_body<float, KB, 256, true, true>(g);
}

}  // namespace

// Eliminate the first n_piv columns of `batch` matrices (see file comment).
// scratch: batch NB x NB block inverses (type T), batch x 2 PERM_STRIDE ints,
// then (256-byte aligned) batch 128 x 128 unit-lower block inverses (type T).
template <class T>
hipError_t lu_eliminate(hipStream_t s, T* W, int batch, long long mat_stride, int ld, int n_piv, int n_rows,
                        int n_cols, int* ipiv, int ipiv_stride, int* status, T* scratch, LuTune tune,
                        hipStream_t s2, hipEvent_t evA, hipEvent_t evF) {
  int* perm = reinterpret_cast<int*>(scratch + (size_t)batch * NB * NB);
  T* Linv = reinterpret_cast<T*>(
      (reinterpret_cast<uintptr_t>(perm + (size_t)batch * 2 * PERM_STRIDE) + 255) & ~uintptr_t(255));
  int* cand0 = reinterpret_cast<int*>(Linv + (size_t)batch * 4 * NB * NB);  // tournament candidates, two rounds
  int* cand1 = cand0 + (size_t)batch * TMAXG * NB;
  LuArgs<T> a{W, mat_stride, ld, n_piv, n_rows, n_cols, ipiv, ipiv_stride, status, perm};
  if (ld % NC != 0) return hipErrorInvalidValue;
  const int rpt = (n_piv + PANEL_THREADS - 1) / PANEL_THREADS;
  // up to 2048 rows: 512 threads, 1..4 rows each; up to 4096: 512 threads with 8
  // rows or 1024 threads with 4 rows; up to 12288: 512 threads, 24 rows each of
  // 4-column sub-panels (register budget)
  const int TPW = tune.tpw;  // 16-row tiles per workgroup (TPW / 4 per wave)
  if (TPW < 4 || TPW % 4) return hipErrorInvalidValue;
  // one-dimensional update grids: at most 2^32 - 1 work-items
  if ((long long)(ld / NC) * ((n_rows + 16 * TPW - 1) / (16 * TPW)) * batch * 256 > 0xffffffffLL)
    return hipErrorInvalidValue;
  const bool tour = tune.panel == 2;
  auto panel = [&](hipStream_t q, int j0, int jb, int lcol0) {
    if (tour) {
      const int g0 = (n_piv - j0 + TR - 1) / TR;
      if (g0 == 1) {
        hipLaunchKernelGGL(k_tslu_final<T>, dim3(batch), dim3(TR), 0, q, a, j0, jb, lcol0, nullptr, 0);
        return;
      }
      hipLaunchKernelGGL(k_tslu_round<T>, dim3(g0, batch), dim3(TR), 0, q, a, j0, jb, nullptr, 0, cand0);
      int n = g0;
      int *in = cand0, *out = cand1;
      while (n > TSETS) {
        const int ng = (n + TSETS - 1) / TSETS;
        hipLaunchKernelGGL(k_tslu_round<T>, dim3(ng, batch), dim3(TR), 0, q, a, j0, jb, in, n, out);
        n = ng;
        std::swap(in, out);
      }
      hipLaunchKernelGGL(k_tslu_final<T>, dim3(batch), dim3(TR), 0, q, a, j0, jb, lcol0, in, n);
      return;
    }
    if (tune.panel == 1 && rpt <= 1)
      hipLaunchKernelGGL((k_panel<T, 1, 1024>), dim3(batch), dim3(1024), 0, q, a, j0, jb, lcol0);
    else if (tune.panel == 1 && rpt <= 4)
      hipLaunchKernelGGL((k_panel<T, 2, 1024>), dim3(batch), dim3(1024), 0, q, a, j0, jb, lcol0);
    else if (rpt <= 1) hipLaunchKernelGGL((k_panel<T, 1, 512>), dim3(batch), dim3(512), 0, q, a, j0, jb, lcol0);
    else if (rpt <= 2) hipLaunchKernelGGL((k_panel<T, 2, 512>), dim3(batch), dim3(512), 0, q, a, j0, jb, lcol0);
    else if (rpt <= 4) hipLaunchKernelGGL((k_panel<T, 4, 512>), dim3(batch), dim3(512), 0, q, a, j0, jb, lcol0);
    // up to 4096 rows: 512 threads with 8 rows of an 8-column sub-panel each,
    // or (wide) 1024 threads with 4 rows (FP64 with 8-column sub-panels: a
    // 16-column FP64 sub-panel of 4 rows does not fit the register budget of
    // 1024 threads)
    else if (n_piv <= 4 * 1024 && tune.panel == 1 && sizeof(T) == 4)
      hipLaunchKernelGGL((k_panel<T, 4, 1024>), dim3(batch), dim3(1024), 0, q, a, j0, jb, lcol0);
    else if (n_piv <= 4 * 1024 && tune.panel == 1)
      hipLaunchKernelGGL((k_panel<T, 4, 1024, 8>), dim3(batch), dim3(1024), 0, q, a, j0, jb, lcol0);
    else if (n_piv <= 4 * 1024)
      hipLaunchKernelGGL((k_panel<T, 8, 512, 8>), dim3(batch), dim3(512), 0, q, a, j0, jb, lcol0);
    else hipLaunchKernelGGL((k_panel<T, 24, 512, 4>), dim3(batch), dim3(512), 0, q, a, j0, jb, lcol0);
  };
  // L of the rows below the pivot rows, A_block U11^{-1}: the non-pivot rows
  // (D), and with the tournament all rows below the block
  auto drows = [&](hipStream_t q, int j0, int jb) {
    const int r0 = tour ? j0 + jb : n_piv;
    if (n_rows <= r0) return;
    hipLaunchKernelGGL(k_uinv<T>, dim3(batch), dim3(NB), 0, q, a, j0, jb, scratch);
    const int ntile = (n_rows - r0 + 15) / 16, ny = (ntile + TPW - 1) / TPW;
    GemmArgs<T> g{W, mat_stride, ld, scratch, (long long)NB * NB, NB, 0, 0, j0, jb, j0, j0, j0 + jb, r0, n_rows,
                  T(1), 0, TPW, 1, ny};
    hipLaunchKernelGGL((k_gemm<T, 64>), dim3((unsigned)(ny * batch)), dim3(256), 0, q, g);
  };
  // A22 -= L21 U12 for the strips [strip0, strip0 + nstrip) with U12 in rows [j0, j0 + K) of W
  auto update = [&](hipStream_t q, int j0, int K, int live0, int strip0, int nstrip, int col_end) {
    if (n_rows <= live0 || nstrip <= 0) return;
    const int ntile = (n_rows - live0 + 15) / 16, ny = (ntile + TPW - 1) / TPW;
    GemmArgs<T> g{W, mat_stride, ld, W, mat_stride, ld, 1, j0, j0, K, strip0, live0, col_end, live0, n_rows,
                  T(-1), 1, TPW, nstrip, ny};
    dim3 grid((unsigned)((long long)nstrip * ny * batch));
    if constexpr (std::is_same<T, float>::value) {
      if (tune.bf16_update) {
        if (K > NB) hipLaunchKernelGGL((k_gemm_bf16<2 * NB>), grid, dim3(256), 0, q, g);
        else hipLaunchKernelGGL((k_gemm_bf16<NB>), grid, dim3(256), 0, q, g);
        return;
      }
    }
    if (K > NB) hipLaunchKernelGGL((k_gemm<T, 2 * NB>), grid, dim3(256), 0, q, g);
    else hipLaunchKernelGGL((k_gemm<T, NB>), grid, dim3(256), 0, q, g);
  };
  if (n_piv > 12 * 1024) return hipErrorInvalidValue;
  // Two streams (s2 given): the factorisation of the next pair of blocks
  // (panels, their non-pivot rows, the pair's own columns) runs on s2 while
  // s finishes the trailing update of the columns beyond the next pair.
  // Event evF hands a factored pair from s2 to s, evA hands the updated
  // next-pair columns (and the free scratch) from s back to s2.  The row
  // swaps of a pair reach the columns right of it only through its k_u12lin
  // on s, after the previous update of those columns, as in the one-stream
  // order.
  const bool split = tune.lookahead && s2 != nullptr && evA != nullptr && evF != nullptr;
  const hipStream_t sm = s, sp = split ? s2 : s;
  hipError_t e;
  auto handoff = [&](hipEvent_t ev, hipStream_t from, hipStream_t to) -> hipError_t {
    if (!split) return hipSuccess;
    hipError_t r = hipEventRecord(ev, from);
    return r == hipSuccess ? hipStreamWaitEvent(to, ev, 0) : r;
  };
  if ((e = handoff(evA, sm, sp)) != hipSuccess) return e;  // fork
  for (int j0 = 0; j0 < n_piv; j0 += 2 * NB) {
    const int jb1 = std::min(NB, n_piv - j0);
    panel(sp, j0, jb1, j0);
    drows(sp, j0, jb1);
    const bool two = (jb1 == NB) && (j0 + NB < n_piv);
    if (!two) {
      if ((e = handoff(evF, sp, sm)) != hipSuccess) return e;
      const int live0 = j0 + jb1, strip0 = live0 / NC * NC;
      const int nstrip = (n_cols > live0) ? (n_cols - strip0 + NC - 1) / NC : 0;
      if (nstrip > 0) {
        hipLaunchKernelGGL(k_u12<T>, dim3(nstrip, batch), dim3(256), 0, sm, a, j0, jb1, strip0, ld);
        update(sm, j0, jb1, live0, strip0, nstrip, ld);
      }
      if ((e = handoff(evA, sm, sp)) != hipSuccess) return e;
      continue;
    }
    // look-ahead: bring the second block's columns up to date with the first
    hipLaunchKernelGGL(k_u12<T>, dim3(1, batch), dim3(256), 0, sp, a, j0, NB, j0 + NB, j0 + NB + std::min(NB, n_piv - (j0 + NB)));
    update(sp, j0, NB, j0 + NB, j0 + NB, 1, j0 + NB + std::min(NB, n_piv - (j0 + NB)));
    const int jb2 = std::min(NB, n_piv - (j0 + NB));
    panel(sp, j0 + NB, jb2, j0);  // also swaps the first block's L columns
    drows(sp, j0 + NB, jb2);
    // both blocks on the remaining strips with one K = 64 + jb2 update
    const int live0 = j0 + NB + jb2, strip0 = live0 / NC * NC;
    const int nstrip = (n_cols > live0) ? (n_cols - strip0 + NC - 1) / NC : 0;
    if (nstrip > 0) hipLaunchKernelGGL(k_linv2<T>, dim3(batch), dim3(256), 0, sp, a, j0, jb2, Linv);
    if ((e = handoff(evF, sp, sm)) != hipSuccess) return e;
    if (nstrip > 0) {
      hipLaunchKernelGGL(k_u12lin<T>, dim3(nstrip, batch), dim3(256), 0, sm, a, j0, jb2, strip0, Linv);
      // the next pair's two strips first, then hand them over
      const int na = (live0 < n_piv && live0 % NC == 0) ? std::min(nstrip, 2) : nstrip;
      update(sm, j0, NB + jb2, live0, strip0, na, ld);
      if ((e = handoff(evA, sm, sp)) != hipSuccess) return e;
      update(sm, j0, NB + jb2, live0, strip0 + na * NC, nstrip - na, ld);
    } else if ((e = handoff(evA, sm, sp)) != hipSuccess) {
      return e;
    }
  }
  if ((e = handoff(evF, sp, sm)) != hipSuccess) return e;  // join
  return hipGetLastError();
}

template hipError_t lu_eliminate<double>(hipStream_t, double*, int, long long, int, int, int, int, int*, int, int*,
                                         double*, LuTune, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t lu_eliminate<float>(hipStream_t, float*, int, long long, int, int, int, int, int*, int, int*,
                                        float*, LuTune, hipStream_t, hipEvent_t, hipEvent_t);

// Elimination scratch of one class: Uinv, permutations and Linv for `batch`
// matrices, in doubles (with room for the 256-byte alignment of Linv).
static size_t class_scratch_doubles(int batch) {
  return (size_t)batch * (NB * NB + 4 * NB * NB + (2 * PERM_STRIDE + 1) / 2 + TMAXG * NB) + 64;
}

// One batched elimination per macro class of chunk j (the chunk's matrices
// of a class are stored consecutively); status flag j * n_classes + k
// belongs to class k of chunk j.  With several classes they run
// concurrently on a few streams (fork from and join back to the context's
// stream), each class with its own scratch slice.  top_only: only the rows
// of S are eliminated (U, L^{-1} P (-C) and L^{-1} P f for the recovery).
// only_class >= 0: that class alone (timing by the autotuner).
hipError_t launch_lu(HdgContext& c, int prec, int chunk, bool top_only, int only_class, bool rhs_only) {
  const int ncl = c.hm.n_classes;
  int* status = reinterpret_cast<int*>(c.ws.small) + (size_t)chunk * ncl;
  const int* cnt = &c.hm.chunk_class_cnt[(size_t)chunk * ncl];
  int nact = 0;
  for (int k = 0; k < ncl; ++k) nact += cnt[k] > 0;
  const int nstreams = nact > 1 ? std::min(nact, 4) : 0;
  hipError_t e;
  if (nstreams > 0 && (int)c.lu_streams.size() < nstreams) {
    for (auto s : c.lu_streams) (void)hipStreamDestroy(s);
    for (auto ev : c.lu_events) (void)hipEventDestroy(ev);
    c.lu_streams.assign(nstreams, nullptr);
    c.lu_events.assign(nstreams + 1, nullptr);
    for (auto& s : c.lu_streams)
      if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return e;
    for (auto& ev : c.lu_events)
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
  }
  // one panel stream and two hand-off events per class slot (look-ahead)
  const int nslots = std::max(nstreams, 1);
  if ((int)c.lu_pstreams.size() < nslots) {
    for (auto s : c.lu_pstreams) (void)hipStreamDestroy(s);
    for (auto ev : c.lu_pevents) (void)hipEventDestroy(ev);
    c.lu_pstreams.assign(nslots, nullptr);
    c.lu_pevents.assign(2 * nslots, nullptr);
    for (auto& s : c.lu_pstreams)
      if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return e;
    for (auto& ev : c.lu_pevents)
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
  }
  if (nstreams > 0) {  // fork
    if ((e = hipEventRecord(c.lu_events[nstreams], c.stream)) != hipSuccess) return e;
    for (int i = 0; i < nstreams; ++i)
      if ((e = hipStreamWaitEvent(c.lu_streams[i], c.lu_events[nstreams], 0)) != hipSuccess) return e;
  }
  // largest classes first (their eliminations take longest)
  std::vector<int> order;
  for (int k = 0; k < ncl; ++k)
    if (cnt[k] > 0) order.push_back(k);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return (double)c.hcs[a].n_u * c.hcs[a].n_u * cnt[a] > (double)c.hcs[b].n_u * c.hcs[b].n_u * cnt[b];
  });
  size_t scr = 0;
  for (size_t i = 0; i < order.size(); ++i) {
    const int k = order[i];
    const HostClass& h = c.hcs[k];
    const size_t ck = (size_t)chunk * ncl + k;
    int* ipiv = c.ws.ipiv + c.hm.class_ipiv_base[k] + (long long)c.hm.chunk_class_rank0[ck] * h.n_u;
    const int batch = cnt[k];
    const int n_rows = top_only ? h.n_u : h.n_rows;
    const int n_cols = (top_only && rhs_only) ? h.n_u + 1 : h.n_cols;
    const int slot = nstreams > 0 ? (int)(i % nstreams) : 0;
    hipStream_t s = nstreams > 0 ? c.lu_streams[slot] : c.stream;
    hipStream_t sp = c.lu_pstreams[slot];
    hipEvent_t evA = c.lu_pevents[2 * slot], evF = c.lu_pevents[2 * slot + 1];
    double* scratch = c.ws.Uinv + scr;
    scr += class_scratch_doubles(batch);
    if (only_class >= 0 && k != only_class) continue;
    LuTune tune = h.tune[prec == 1 ? 1 : 0];
    tune.bf16_update = (prec == 1 && c.bf16_update && !top_only) ? 1 : 0;
    if (prec == 1)
      e = lu_eliminate<float>(s, reinterpret_cast<float*>(c.ws.Wm) + c.hm.chunk_class_w[ck], batch, h.wstride, h.ldw,
                              h.n_u, n_rows, n_cols, ipiv, h.n_u, status + k, reinterpret_cast<float*>(scratch),
                              tune, sp, evA, evF);
    else
      e = lu_eliminate<double>(s, c.ws.Wm + c.hm.chunk_class_w[ck], batch, h.wstride, h.ldw, h.n_u, n_rows, n_cols,
                               ipiv, h.n_u, status + k, scratch, tune, sp, evA, evF);
    if (e != hipSuccess) return e;
  }
  if (nstreams > 0) {  // join
    for (int i = 0; i < nstreams; ++i) {
      if ((e = hipEventRecord(c.lu_events[i], c.lu_streams[i])) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(c.stream, c.lu_events[i], 0)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

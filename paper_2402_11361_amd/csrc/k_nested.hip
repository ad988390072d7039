// Nested hybridisation inside a macro: a third static-condensation layer (an
// alternative local structure to the C0 macro of the paper's Sec. 2.2).
//
// On a mesh of one element per macro every element is hybridised on its own
// and the second-layer condensation leaves the element blocks A-hat^{T_e},
// b-hat^{T_e} (eq. C44 pieces).  Grouping the elements into blocks of M per
// axis, each block assembles its elements' blocks over the faces of its
// elements, internal faces first, and eliminates their traces (eq. ASC2 once
// more, with the same batched elimination as the macros):
//   W_G = [[A_II, A_IB, b_I], [A_BI, A_BB, b_B]]  ->  A-hat^G = A_BB - A_BI A_II^{-1} A_IB,
//                                                      b-hat^G = b_B - A_BI A_II^{-1} b_I.
// Block-local trace order: internal faces in increasing global face id, then
// boundary faces likewise, each face's unknowns in their global order.
#include "context.h"
#include <algorithm>
#include <set>

template <class T>
hipError_t lu_eliminate(hipStream_t s, T* W, int batch, long long mat_stride, int ld, int n_piv, int n_rows,
                        int n_cols, int* ipiv, int ipiv_stride, int* status, T* scratch, LuTune tune,
                        hipStream_t s2, hipEvent_t evA, hipEvent_t evF);

struct NestedPlan {
  int block_m = 0, n_blocks = 0, n_el = 0, nb_e = 0, n_I = 0, n_B = 0, ld = 0, rows = 0;
  long long wstride = 0;
  int* elem = nullptr;   // [n_blocks][n_el] macro ids
  int* map = nullptr;    // [n_blocks][n_el][nb_e] block-local index of each element trace unknown
  double* W = nullptr;   // [n_blocks] tiled block matrices
  int* ipiv = nullptr;   // [n_blocks][n_I]
  int* status = nullptr;
  double* scratch = nullptr;
  // block skeleton: its faces in increasing face id, each face's unknowns in order
  long long n_skel = 0;
  int* skel_idx = nullptr;        // [n_blocks][n_B] skeleton index of each boundary unknown of a block
  int* owners = nullptr;          // [n_skel][2] g n_B + r of the (one or two) blocks holding it, lower block first; -1 = none
  long long* skel_glob = nullptr; // [n_skel] element-trace index of each skeleton unknown
  long long* int_glob = nullptr;  // [n_blocks][n_I] element-trace index of each internal unknown
  double* ypart = nullptr;        // [n_blocks][n_B] per-block products
  double* diag = nullptr;         // [n_skel] diagonal of the assembled skeleton operator
  double* xint = nullptr;         // [n_blocks][n_I] internal traces
  double* bskel = nullptr;        // [n_skel]
  double* xskel = nullptr;        // [n_skel]
  bool condensed = false;         // the block matrices hold the last hdg_condense_nested
  ~NestedPlan() {
    for (void* p : {(void*)elem, (void*)map, (void*)W, (void*)ipiv, (void*)status, (void*)scratch, (void*)skel_idx,
                    (void*)owners, (void*)skel_glob, (void*)int_glob, (void*)ypart, (void*)diag, (void*)xint,
                    (void*)bskel, (void*)xskel})
      if (p) (void)hipFree(p);
  }
};

namespace {

// element block entry (r, k) and b-hat entry r of macro e after an FP64
// condensation: compact copies when chunked, else the corner of the tiled W
__device__ __forceinline__ double elem_ahat(const MeshDev& md, const double* Wm, const double* Ac, int chunked,
                                            int e, int nu, int ldw, int nb, int r, int k) {
  if (chunked) return Ac[md.a32_off[e] + (long long)r * nb + k];
  return Wm[md.w_off[e] + wtix(nu + r, nu + k, ldw)];
}

// One workgroup per (block, element): the element's A-hat and b-hat added
// into the block matrix.  At most two elements add to one entry (the two
// sides of a face), and 0 + a + b = 0 + b + a, so the sums do not depend on
// the order of the atomic additions.
__global__ void __launch_bounds__(256) k_nested_form(MeshDev md, const double* __restrict__ Wm,
                                                     const double* __restrict__ Ac, const double* __restrict__ bloc,
                                                     int chunked, int nu, int ldw, int ncols_e, const int* __restrict__ elem,
                                                     const int* __restrict__ map, int n_el, int nb, int rhs_col, int ld,
                                                     long long wstride, double* __restrict__ Wn) {
  const int g = blockIdx.x / n_el, j = blockIdx.x % n_el;
  const int e = elem[(size_t)g * n_el + j];
  const int* mp = map + ((size_t)g * n_el + j) * nb;
  double* Wg = Wn + (size_t)g * wstride;
  for (int x = threadIdx.x; x < nb * nb; x += blockDim.x) {
    const int r = x / nb, k = x % nb;
    atomicAdd(&Wg[wtix(mp[r], mp[k], ld)], elem_ahat(md, Wm, Ac, chunked, e, nu, ldw, nb, r, k));
  }
  for (int r = threadIdx.x; r < nb; r += blockDim.x) {
    const double b = chunked ? bloc[md.b_off[e] + r] : Wm[md.w_off[e] + wtix(nu + r, ncols_e - 1, ldw)];
    atomicAdd(&Wg[wtix(mp[r], rhs_col, ld)], b);
  }
}

// A-hat^G and b-hat^G out of the eliminated block matrices
__global__ void k_nested_extract(const double* __restrict__ Wn, long long wstride, int ld, int nI, int nB, int n_blocks,
                                 double* __restrict__ ahat, double* __restrict__ bhat) {
  const long long per = (long long)nB * (nB + 1), total = per * n_blocks;
  for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < total;
       x += (long long)gridDim.x * blockDim.x) {
    const int g = (int)(x / per), y = (int)(x % per), r = y / (nB + 1), k = y % (nB + 1);
    const double v = Wn[(size_t)g * wstride + wtix(nI + r, nI + k, ld)];
    if (k < nB) ahat[((size_t)g * nB + r) * nB + k] = v;
    else bhat[(size_t)g * nB + r] = v;
  }
}

__device__ __forceinline__ double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int NROWS = 16;  // rows of a block matrix per workgroup in the products

// ypart[g][r] = sum_k A-hat^G[r][k] x[skel_idx[g][k]] for the rows of this
// workgroup (the block's x_B staged in LDS; one wave per row, 4 rows each).
__global__ void __launch_bounds__(256) k_nested_apply_part(const double* __restrict__ Wn, long long wstride, int ld,
                                                           int nI, int nB, const int* __restrict__ skel_idx,
                                                           const double* __restrict__ x, double* __restrict__ ypart) {
  extern __shared__ double xs[];
  const int g = blockIdx.x, r0 = blockIdx.y * NROWS;
  const int* si = skel_idx + (size_t)g * nB;
  for (int k = threadIdx.x; k < nB; k += blockDim.x) xs[k] = x[si[k]];
  __syncthreads();
  const double* Wg = Wn + (size_t)g * wstride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int rr = wave; rr < NROWS; rr += 4) {
    const int r = r0 + rr;
    if (r >= nB) break;
    double s = 0.0;
    for (int k = lane; k < nB; k += 64) s += Wg[wtix(nI + r, nI + k, ld)] * xs[k];
    s = wave_sum64(s);
    if (lane == 0) ypart[(size_t)g * nB + r] = s;
  }
}

// y[s] = sum over the owners of skeleton unknown s of their entries of
// src[g n_B + r] (fixed order: lower block first)
__global__ void k_nested_owner_sum(long long n_skel, const int* __restrict__ owners, const double* __restrict__ src,
                                   double* __restrict__ y) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n_skel; s += (long long)gridDim.x * blockDim.x) {
    const int o0 = owners[2 * s], o1 = owners[2 * s + 1];
    double v = src[o0];
    if (o1 >= 0) v += src[o1];
    y[s] = v;
  }
}

// per block boundary unknown: the diagonal of A-hat^G and b-hat^G (for the
// owner sums of the skeleton diagonal and right-hand side)
__global__ void k_nested_diag_rhs(const double* __restrict__ Wn, long long wstride, int ld, int nI, int nB, int n_blocks,
                                  double* __restrict__ dpart, double* __restrict__ bpart) {
  const long long total = (long long)n_blocks * nB;
  for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < total; x += (long long)gridDim.x * blockDim.x) {
    const int g = (int)(x / nB), r = (int)(x % nB);
    const double* Wg = Wn + (size_t)g * wstride;
    dpart[x] = Wg[wtix(nI + r, nI + r, ld)];
    bpart[x] = Wg[wtix(nI + r, nI + nB, ld)];
  }
}

__global__ void k_nested_jacobi(long long n, const double* __restrict__ diag, const double* __restrict__ v,
                                double* __restrict__ z) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n; s += (long long)gridDim.x * blockDim.x)
    z[s] = diag[s] != 0.0 ? v[s] / diag[s] : v[s];
}

// Recovery right-hand side of the internal traces after the elimination of
// block g (rows [0, n_I) hold U | L^{-1} P A_IB | L^{-1} P b_I):
// xint[g][i] = (L^{-1} P b_I)_i - sum_k (L^{-1} P A_IB)_ik x_B[k].
__global__ void __launch_bounds__(256) k_nested_rec_rhs(const double* __restrict__ Wn, long long wstride, int ld,
                                                        int nI, int nB, const int* __restrict__ skel_idx,
                                                        const double* __restrict__ xskel, double* __restrict__ xint) {
  extern __shared__ double xs[];
  const int g = blockIdx.x, r0 = blockIdx.y * NROWS;
  const int* si = skel_idx + (size_t)g * nB;
  for (int k = threadIdx.x; k < nB; k += blockDim.x) xs[k] = xskel[si[k]];
  __syncthreads();
  const double* Wg = Wn + (size_t)g * wstride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int rr = wave; rr < NROWS; rr += 4) {
    const int r = r0 + rr;
    if (r >= nI) break;
    double s = 0.0;
    for (int k = lane; k < nB; k += 64) s += Wg[wtix(r, nI + k, ld)] * xs[k];
    s = wave_sum64(s);
    if (lane == 0) xint[(size_t)g * nI + r] = Wg[wtix(r, nI + nB, ld)] - s;
  }
}

// x = U^{-1} xint in place for block g: 64-row blocks from the bottom, the
// rows' products with the solved part by one wave each, the 64 x 64
// triangle by wave 0 in registers.
__global__ void __launch_bounds__(256) k_nested_rec_trsv(const double* __restrict__ Wn, long long wstride, int ld,
                                                         int nI, double* __restrict__ xint) {
  __shared__ double sU[64][65];
  __shared__ double sz[64];
  const int g = blockIdx.x;
  const double* U = Wn + (size_t)g * wstride;
  double* x = xint + (size_t)g * nI;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nblk = (nI + 63) / 64;
  for (int b = nblk - 1; b >= 0; --b) {
    const int i0 = b * 64, i1 = min(nI, i0 + 64), nr = i1 - i0;
    for (int rr = wave; rr < nr; rr += 4) {
      const int r = i0 + rr;
      double s = 0.0;
      for (int c = i1 + lane; c < nI; c += 64) s += U[wtix(r, c, ld)] * x[c];
      s = wave_sum64(s);
      if (lane == 0) sz[rr] = x[r] - s;
    }
    for (int i = threadIdx.x; i < nr * nr; i += blockDim.x) {
      const int r = i / nr, c = i % nr;
      sU[r][c] = U[wtix(i0 + r, i0 + c, ld)];
    }
    __syncthreads();
    if (wave == 0) {
      double xv = (lane < nr) ? sz[lane] : 0.0;
      for (int r = nr - 1; r >= 0; --r) {
        double s = (lane > r && lane < nr) ? sU[r][lane] * xv : 0.0;
        s = wave_sum64(s);
        if (lane == r) xv = (xv - s) / sU[r][r];
      }
      if (lane < nr) x[i0 + lane] = xv;
    }
    __syncthreads();
  }
}

// the element-trace vector from the skeleton and internal traces
__global__ void k_nested_scatter(long long n_skel, const long long* __restrict__ skel_glob,
                                 const double* __restrict__ xskel, long long n_int, const long long* __restrict__ int_glob,
                                 const double* __restrict__ xint, double* __restrict__ xfull) {
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n_skel; s += st) xfull[skel_glob[s]] = xskel[s];
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n_int; s += st) xfull[int_glob[s]] = xint[s];
}

inline unsigned grid_n(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 65535)); }

}  // namespace

// Block structure for blocks of M elements per axis; "" on success.
std::string nested_plan(HdgContext& c, int M, std::shared_ptr<NestedPlan>& out) {
  const HostMesh& hm = c.hm;
  const int d = hm.dim;
  if (M < 1) return "block size must be positive";
  if (hm.n_classes != 1) return "nested blocks need macros of one shape";
  for (int k = 0; k < d; ++k) {
    if (c.hcs[0].m[k] != 1) return "nested blocks need one element per macro";
    if (hm.n_seg[k] % M) return "the element count per axis must be a multiple of the block size";
    if (hm.periodic[k] && hm.n_seg[k] < 2) return "a periodic axis of one element gives a face with itself";
  }
  auto P = std::make_shared<NestedPlan>();
  P->block_m = M;
  int nblk[3] = {1, 1, 1};
  for (int k = 0; k < d; ++k) nblk[k] = hm.n_seg[k] / M;
  P->n_blocks = nblk[0] * nblk[1] * nblk[2];
  {
    int ne = 1;
    for (int k = 0; k < d; ++k) ne *= M;
    P->n_el = ne;
  }
  P->nb_e = c.hcs[0].n_b;
  std::vector<int> block_of(hm.n_macros), seen(P->n_blocks, 0);
  std::vector<int> elem((size_t)P->n_blocks * P->n_el);
  for (int i = 0; i < hm.n_macros; ++i) {
    int t = i, g = 0, mul = 1;
    for (int k = 0; k < d; ++k) {
      const int s = t % hm.n_seg[k];
      t /= hm.n_seg[k];
      g += (s / M) * mul;
      mul *= nblk[k];
    }
    block_of[i] = g;
    elem[(size_t)g * P->n_el + seen[g]++] = i;  // increasing macro index
  }
  std::vector<int> map((size_t)P->n_blocks * P->n_el * P->nb_e);
  std::vector<std::vector<int>> blk_inner(P->n_blocks), blk_bnd(P->n_blocks);
  for (int g = 0; g < P->n_blocks; ++g) {
    std::set<int> fs;
    for (int j = 0; j < P->n_el; ++j)
      for (int lf = 0; lf < 2 * d; ++lf) fs.insert(hm.macro_face[(size_t)elem[(size_t)g * P->n_el + j] * 2 * d + lf]);
    std::vector<int> inner, bnd;
    for (int F : fs) {
      const int mi = hm.face_minus[F], pl = hm.face_plus[F];
      if (mi >= 0 && pl >= 0 && block_of[mi] == g && block_of[pl] == g) inner.push_back(F);
      else bnd.push_back(F);
    }
    std::vector<long long> loc(hm.n_faces, -1);
    long long pos = 0, nI = 0;
    for (int F : inner) { loc[F] = pos; pos += hm.face_ndof[F]; }
    nI = pos;
    for (int F : bnd) { loc[F] = pos; pos += hm.face_ndof[F]; }
    if (g == 0) { P->n_I = (int)nI; P->n_B = (int)(pos - nI); }
    else if (P->n_I != nI || P->n_B != pos - nI) return "blocks with different face counts";
    blk_inner[g] = inner;
    blk_bnd[g] = bnd;
    for (int j = 0; j < P->n_el; ++j) {
      const int e = elem[(size_t)g * P->n_el + j];
      int r = 0;
      for (int lf = 0; lf < 2 * d; ++lf) {
        const int F = hm.macro_face[(size_t)e * 2 * d + lf];
        for (int q = 0; q < hm.face_ndof[F]; ++q)
          map[((size_t)g * P->n_el + j) * P->nb_e + r++] = (int)(loc[F] + q);
      }
      if (r != P->nb_e) return "element trace size mismatch";
    }
  }
  // skeleton: faces that are internal to no block, in increasing face id
  std::vector<char> is_inner(hm.n_faces, 0);
  for (const auto& v : blk_inner)
    for (int F : v) is_inner[F] = 1;
  std::vector<long long> skel_off(hm.n_faces, -1);
  std::vector<long long> skel_glob, int_glob;
  for (int F = 0; F < hm.n_faces; ++F) {
    if (is_inner[F]) continue;
    skel_off[F] = (long long)skel_glob.size();
    for (int q = 0; q < hm.face_ndof[F]; ++q) skel_glob.push_back(hm.face_off[F] + q);
  }
  P->n_skel = (long long)skel_glob.size();
  std::vector<int> skel_idx((size_t)P->n_blocks * P->n_B), owners((size_t)2 * P->n_skel, -1);
  for (int g = 0; g < P->n_blocks; ++g) {
    int r = 0;
    for (int F : blk_bnd[g])
      for (int q = 0; q < hm.face_ndof[F]; ++q, ++r) {
        const long long sidx = skel_off[F] + q;
        skel_idx[(size_t)g * P->n_B + r] = (int)sidx;
        int* o = &owners[(size_t)2 * sidx];
        if (o[0] < 0) o[0] = g * P->n_B + r;
        else if (o[1] < 0) o[1] = g * P->n_B + r;
        else return "a skeleton face bordered by more than two blocks";
      }
    for (int F : blk_inner[g])
      for (int q = 0; q < hm.face_ndof[F]; ++q) int_glob.push_back(hm.face_off[F] + q);
  }
  for (long long s2 = 0; s2 < P->n_skel; ++s2)
    if (owners[(size_t)2 * s2] < 0) return "a skeleton face without a block";
  if ((long long)P->n_blocks * P->n_B >= (1LL << 31)) return "too many block boundary unknowns";
  const int n = P->n_I + P->n_B;
  if (P->n_I > 12 * 1024) return "more internal-face unknowns per block than the elimination takes";
  if (P->n_B > 8 * 1024) return "more boundary unknowns per block than the skeleton products stage";
  P->ld = (n + 1 + 63) / 64 * 64;
  P->rows = (n + 15) / 16 * 16;
  P->wstride = (long long)P->rows * P->ld;
  auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 8) == hipSuccess; };
  const size_t scr = (size_t)P->n_blocks * (64 * 64 + 128 * 128 + 512 + 48 * 64) + 64;
  if (!alloc((void**)&P->elem, sizeof(int) * elem.size()) || !alloc((void**)&P->map, sizeof(int) * map.size()) ||
      !alloc((void**)&P->W, sizeof(double) * (size_t)P->n_blocks * P->wstride) ||
      !alloc((void**)&P->ipiv, sizeof(int) * (size_t)P->n_blocks * std::max(P->n_I, 1)) ||
      !alloc((void**)&P->status, sizeof(int)) || !alloc((void**)&P->scratch, sizeof(double) * scr) ||
      !alloc((void**)&P->skel_idx, sizeof(int) * skel_idx.size()) ||
      !alloc((void**)&P->owners, sizeof(int) * owners.size()) ||
      !alloc((void**)&P->skel_glob, sizeof(long long) * skel_glob.size()) ||
      !alloc((void**)&P->int_glob, sizeof(long long) * int_glob.size()) ||
      !alloc((void**)&P->ypart, sizeof(double) * skel_idx.size()) ||
      !alloc((void**)&P->diag, sizeof(double) * std::max<size_t>(skel_idx.size(), (size_t)P->n_skel)) ||
      !alloc((void**)&P->xint, sizeof(double) * int_glob.size()) ||
      !alloc((void**)&P->bskel, sizeof(double) * std::max<size_t>(skel_idx.size(), (size_t)P->n_skel)) ||
      !alloc((void**)&P->xskel, sizeof(double) * P->n_skel))
    return "out of device memory for the nested blocks";
  if (hipMemcpy(P->elem, elem.data(), sizeof(int) * elem.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->skel_idx, skel_idx.data(), sizeof(int) * skel_idx.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->owners, owners.data(), sizeof(int) * owners.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->skel_glob, skel_glob.data(), sizeof(long long) * skel_glob.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      (!int_glob.empty() &&
       hipMemcpy(P->int_glob, int_glob.data(), sizeof(long long) * int_glob.size(), hipMemcpyHostToDevice) != hipSuccess))
    return "upload of the block maps failed";
  out = P;
  return "";
}

// Third-layer condensation of every block; *singular receives the first
// singular block + 1 (0 = none) after the stream has been synchronised.
hipError_t launch_condense_nested(HdgContext& c, NestedPlan& P, double* ahat, double* bhat, int* singular) {
  const HostClass& h = c.hcs[0];
  const int n = P.n_I + P.n_B;
  hipError_t e;
  if ((e = hipMemsetAsync(P.W, 0, sizeof(double) * (size_t)P.n_blocks * P.wstride, c.stream)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(P.status, 0, sizeof(int), c.stream)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_nested_form, dim3((unsigned)(P.n_blocks * P.n_el)), dim3(256), 0, c.stream, c.md, c.ws.Wm,
                     c.ws.Ac, c.ws.bloc, c.hm.chunked() ? 1 : 0, h.n_u, h.ldw, h.n_cols, P.elem, P.map, P.n_el,
                     P.nb_e, n, P.ld, P.wstride, P.W);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (P.n_I > 0) {
    LuTune t;  // tournament pivoting, one stream
    t.tpw = 32;
    t.panel = 2;
    t.lookahead = 0;
    if ((e = lu_eliminate<double>(c.stream, P.W, P.n_blocks, P.wstride, P.ld, P.n_I, n, n + 1, P.ipiv, P.n_I,
                                  P.status, P.scratch, t, nullptr, nullptr, nullptr)) != hipSuccess)
      return e;
  }
  const long long total = (long long)P.n_blocks * P.n_B * (P.n_B + 1);
  hipLaunchKernelGGL(k_nested_extract, dim3((unsigned)std::min<long long>((total + 255) / 256, 65535)), dim3(256), 0,
                     c.stream, P.W, P.wstride, P.ld, P.n_I, P.n_B, P.n_blocks, ahat, bhat);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // skeleton diagonal (Jacobi preconditioner) and right-hand side: owner sums
  // of the blocks' diagonals and b-hat^G (parts staged in ypart and bskel)
  const long long nbb = (long long)P.n_blocks * P.n_B;
  hipLaunchKernelGGL(k_nested_diag_rhs, dim3(grid_n(nbb)), dim3(256), 0, c.stream, P.W, P.wstride, P.ld, P.n_I, P.n_B,
                     P.n_blocks, P.ypart, P.bskel);
  hipLaunchKernelGGL(k_nested_owner_sum, dim3(grid_n(P.n_skel)), dim3(256), 0, c.stream, P.n_skel, P.owners, P.ypart,
                     P.diag);
  hipLaunchKernelGGL(k_nested_owner_sum, dim3(grid_n(P.n_skel)), dim3(256), 0, c.stream, P.n_skel, P.owners, P.bskel,
                     P.xskel);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(P.bskel, P.xskel, sizeof(double) * P.n_skel, hipMemcpyDeviceToDevice, c.stream)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(singular, P.status, sizeof(int), hipMemcpyDeviceToHost, c.stream)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(c.stream)) != hipSuccess) return e;
  P.condensed = (*singular == 0);
  return hipSuccess;
}

// y = sum_G P_G^T A-hat^G P_G x on the block skeleton (deterministic: per-block
// products, then the owner sums)
hipError_t launch_nested_apply(HdgContext& c, NestedPlan& P, const double* x, double* y) {
  const dim3 grid((unsigned)P.n_blocks, (unsigned)((P.n_B + NROWS - 1) / NROWS));
  hipLaunchKernelGGL(k_nested_apply_part, grid, dim3(256), sizeof(double) * P.n_B, c.stream, P.W, P.wstride, P.ld, P.n_I,
                     P.n_B, P.skel_idx, x, P.ypart);
  hipLaunchKernelGGL(k_nested_owner_sum, dim3(grid_n(P.n_skel)), dim3(256), 0, c.stream, P.n_skel, P.owners, P.ypart, y);
  return hipGetLastError();
}

// z = D^{-1} v with D the diagonal of the skeleton operator
hipError_t launch_nested_jacobi(HdgContext& c, NestedPlan& P, const double* v, double* z) {
  hipLaunchKernelGGL(k_nested_jacobi, dim3(grid_n(P.n_skel)), dim3(256), 0, c.stream, P.n_skel, P.diag, v, z);
  return hipGetLastError();
}

// the element-trace vector: skeleton traces in place, internal traces
// x_I = U^{-1} (L^{-1} P b_I - L^{-1} P A_IB x_B) block by block
hipError_t launch_nested_recover(HdgContext& c, NestedPlan& P, const double* xskel, double* xfull) {
  if (P.n_I > 0) {
    const dim3 grid((unsigned)P.n_blocks, (unsigned)((P.n_I + NROWS - 1) / NROWS));
    hipLaunchKernelGGL(k_nested_rec_rhs, grid, dim3(256), sizeof(double) * P.n_B, c.stream, P.W, P.wstride, P.ld, P.n_I,
                       P.n_B, P.skel_idx, xskel, P.xint);
    hipLaunchKernelGGL(k_nested_rec_trsv, dim3((unsigned)P.n_blocks), dim3(256), 0, c.stream, P.W, P.wstride, P.ld,
                       P.n_I, P.xint);
  }
  const long long n_int = (long long)P.n_blocks * P.n_I;
  hipLaunchKernelGGL(k_nested_scatter, dim3(grid_n(std::max(P.n_skel, n_int))), dim3(256), 0, c.stream, P.n_skel,
                     P.skel_glob, xskel, n_int, P.int_glob, P.xint, xfull);
  return hipGetLastError();
}

long long nested_skeleton_size(const NestedPlan& P) { return P.n_skel; }
bool nested_condensed(const NestedPlan& P) { return P.condensed; }
double* nested_rhs(NestedPlan& P) { return P.bskel; }
double* nested_xskel(NestedPlan& P) { return P.xskel; }

void nested_dims(const NestedPlan& P, int* n_blocks, int* n_internal, int* n_boundary) {
  if (n_blocks) *n_blocks = P.n_blocks;
  if (n_internal) *n_internal = P.n_I;
  if (n_boundary) *n_boundary = P.n_B;
}

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
  ~NestedPlan() {
    for (void* p : {(void*)elem, (void*)map, (void*)W, (void*)ipiv, (void*)status, (void*)scratch})
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
  const int n = P->n_I + P->n_B;
  if (P->n_I > 12 * 1024) return "more internal-face unknowns per block than the elimination takes";
  P->ld = (n + 1 + 63) / 64 * 64;
  P->rows = (n + 15) / 16 * 16;
  P->wstride = (long long)P->rows * P->ld;
  auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 8) == hipSuccess; };
  const size_t scr = (size_t)P->n_blocks * (64 * 64 + 128 * 128 + 512 + 48 * 64) + 64;
  if (!alloc((void**)&P->elem, sizeof(int) * elem.size()) || !alloc((void**)&P->map, sizeof(int) * map.size()) ||
      !alloc((void**)&P->W, sizeof(double) * (size_t)P->n_blocks * P->wstride) ||
      !alloc((void**)&P->ipiv, sizeof(int) * (size_t)P->n_blocks * std::max(P->n_I, 1)) ||
      !alloc((void**)&P->status, sizeof(int)) || !alloc((void**)&P->scratch, sizeof(double) * scr))
    return "out of device memory for the nested blocks";
  if (hipMemcpy(P->elem, elem.data(), sizeof(int) * elem.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice) != hipSuccess)
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
  if ((e = hipMemcpyAsync(singular, P.status, sizeof(int), hipMemcpyDeviceToHost, c.stream)) != hipSuccess) return e;
  return hipStreamSynchronize(c.stream);
}

void nested_dims(const NestedPlan& P, int* n_blocks, int* n_internal, int* n_boundary) {
  if (n_blocks) *n_blocks = P.n_blocks;
  if (n_internal) *n_internal = P.n_I;
  if (n_boundary) *n_boundary = P.n_B;
}

// Formation of the per-macro augmented matrix of the second-layer
// condensation (paper eq. AP12, ASC2a/b):
//     W = [[ S, -C, f ],      S = A_uu - A_uq A_qq^{-1} A_qu
//          [ D,  E, g ]]      C = -A_u,uh + A_uq A_qq^{-1} A_q,uh
//                             f = A_uq A_qq^{-1} R_Q - R_U
//                             D = A_uh,u - A_uh,q A_qq^{-1} A_qu
//                             E = A_uh,uh - A_uh,q A_qq^{-1} A_q,uh
//                             g = -R_Uh + A_uh,q A_qq^{-1} R_Q
// Eliminating the first n_u columns of W (with partial pivoting in the S
// rows) leaves A-hat^{T_i} = E + D S^{-1} C and b-hat^{T_i} = g - D S^{-1} f in
// the bottom-right corner.
//
// A_qq^{-1} A_qu and A_qq^{-1} A_q,uh are never formed: on a box macro the mass
// matrix is the tensor product of 1D masses, so per direction k
//   A_qq^{-1} A_qu   = I (x) C_k with C_k = M_k^{-1} B_k acting along axis k,
//   A_qq^{-1} A_q,uh = -(I (x) M^{-1} E_k), whose columns for the face (k, s)
//                      are sign_s M_k^{-1}[:, end_s] along axis k times the
//                      identity on the tangential node indices.
// One workgroup builds the NR rows of one group (NR = n_s: the rows of the
// n_s components of one node, which share every target index; NR = 1 for
// classes whose n_s rows do not fit in LDS); contributions are added element
// by element (and direction by direction) into LDS row buffers, in a fixed
// order.
#include "context.h"
#include <cstdio>

namespace {


struct FormPtrs {
  const double *AUU, *AUQ, *SUB, *RU, *RQt, *RBloc;
  double* gloc;  // non-null: g goes here in FP64 and its W entries are 0
  int nsA, dnsA, sub_stride, off_AUB, off_ABU, off_ABQ, off_ABB;
  long long group0;  // first row group of the launch (groups of all macros numbered consecutively)
  int coef_off;      // LDS offset (doubles) of the staged coefficient rows, after the row buffers
  int only_class;    // >= 0: rows of other macro classes are skipped
  int split_cols;    // >= 0: grouped launch takes classes with n_cols <= split_cols, single-row launch the rest
  int tab_off;       // LDS byte offset of the class's 1D operators C1D and Minv1D (FP64)
  // non-null: recovery form (the S rows only, for the local recovery after a
  // chunked condensation): the right-hand side f + C duhat of eq. Csc4a goes
  // to column n_u and the row is stored up to the end of that column's strip
  const double* duhat;
};

// Macro of row group G: a guess from the mean group count per macro (exact
// when every macro has the same size), else the binary search.
__device__ __forceinline__ int macro_of_row(const long long* off, int n, long long g) {
  int i = (int)((double)g / (double)off[n] * n);
  i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
  if (off[i] <= g && g < off[i + 1]) return i;
  return find_in(off, n, g);
}

// Quotient and remainder of 0 <= x < 2^22 by 1 <= y < 2^22 through the FP32
// reciprocal: the relative error of x * rcp(y) is below 2^-22, so the
// truncated quotient is off by at most one and one correction makes it exact.
__device__ __forceinline__ int2 divmod(int x, int y) {
  int q = (int)((float)x * __builtin_amdgcn_rcpf((float)y));
  int r = x - q * y;
  if (r < 0) { --q; r += y; } else if (r >= y) { ++q; r -= y; }
  return make_int2(q, r);
}

__device__ __forceinline__ void digits(int x, int base, int d, int* out) {
  for (int k = 0; k < d; ++k) { const int2 qr = divmod(x, base); out[k] = qr.y; x = qr.x; }
}

// Adds, for direction k, the contributions of NR coefficient rows
// coef(rr, k, cp, b) (element-local nodes b of element e) through
//   line targets  row_rr[cp*N + node(b with b_k -> n_k)] += sgn_line * sum_bk coef * C1D_k[e_k p + b_k][n_k]
//   face targets  row_rr[n_u + nf_off[2k+s] + cp*nf + j(b_tan)] += sgn_face * sign_s * sum_bk coef * Minv_k[e_k p + b_k][end_s]
// (row_rr = row + rr * ldr).  The coefficient functor returns 0 for element
// nodes that carry none (trace rows use only the nodes of their sub-face).
template <int NR, int NT, class TL, class Coef>
__device__ void add_direction(const ClassDev& cd, const double* C1Ds, const double* Minv1Ds, int e, int k, Coef coef,
                              double sgn_line, double sgn_face, TL* row, int ldr, int tid) {
  const int d = cd.dim, p = cd.p, A1 = p + 1, ns = cd.ns;
  int eidx[3] = {0, 0, 0};
  {
    int t = e;
    for (int j = 0; j < d; ++j) { const int2 qr = divmod(t, cd.m[j]); eidx[j] = qr.y; t = qr.x; }
  }
  const int nk = cd.n1[k], nm = cd.nmax1;
  const int T = cd.T;  // (p+1)^(d-1) tangential combinations of an element
  const double* Ck = C1Ds + (size_t)k * nm * nm;     // LDS copies of cd.C1D, cd.Minv1D
  const double* Mk = Minv1Ds + (size_t)k * nm * nm;
  int stride[3] = {1, cd.n1[0], cd.n1[0] * cd.n1[1]};
  // line targets
  for (int i = tid; i < ns * T * nk; i += NT) {
    const int2 q1 = divmod(i, T * nk), q2 = divmod(q1.y, nk);
    const int cp = q1.x, t = q2.x, n = q2.y;
    int td[2] = {0, 0};
    digits(t, A1, d - 1, td);
    int bd[3] = {0, 0, 0}, ti = 0;
    for (int j = 0; j < d; ++j) if (j != k) bd[j] = td[ti++];
    double s[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) s[rr] = 0.0;
    int node0 = 0;
    for (int j = 0; j < d; ++j) if (j != k) node0 += (eidx[j] * p + bd[j]) * stride[j];
    for (int bk = 0; bk < A1; ++bk) {
      bd[k] = bk;
      const int b = bd[0] + A1 * (bd[1] + A1 * bd[2]);
      const double ck = Ck[(eidx[k] * p + bk) * nm + n];
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) s[rr] += coef(rr, k, cp, b) * ck;
    }
    const int col = cp * cd.N + node0 + n * stride[k];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) row[rr * ldr + col] += (TL)(sgn_line * s[rr]);
  }
  // face targets on the two macro faces normal to k
  for (int i = tid; i < 2 * ns * T; i += NT) {
    const int2 q1 = divmod(i, ns * T), q2 = divmod(q1.y, T);
    const int sidx = q1.x, cp = q2.x, t = q2.y;
    int td[2] = {0, 0};
    digits(t, A1, d - 1, td);
    int bd[3] = {0, 0, 0}, ti = 0;
    for (int j = 0; j < d; ++j) if (j != k) bd[j] = td[ti++];
    const int end = (sidx == 0) ? 0 : nk - 1;
    const double sgn = (sidx == 0) ? -1.0 : 1.0;
    double s[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) s[rr] = 0.0;
    for (int bk = 0; bk < A1; ++bk) {
      bd[k] = bk;
      const int b = bd[0] + A1 * (bd[1] + A1 * bd[2]);
      const double mk = Mk[(eidx[k] * p + bk) * nm + end];
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) s[rr] += coef(rr, k, cp, b) * mk;
    }
    // trace node id on face (k, sidx): tangential macro coordinates, lower axis fastest
    int j = 0, mul = 1;
    for (int a = 0; a < d; ++a) {
      if (a == k) continue;
      j += (eidx[a] * p + bd[a]) * mul;
      mul *= cd.n1[a];
    }
    const int lf = 2 * k + sidx;
    const int col = cd.n_u + cd.nf_off[lf] + cp * cd.nf_nodes[lf] + j;
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) row[rr * ldr + col] += (TL)(sgn_face * sgn * s[rr]);
  }
}

// Sum over the workgroup of NR per-thread values (wave shuffles, then LDS).
template <int NR, int NT>
__device__ void block_sum(double* v, double* red, int tid) {
#pragma unroll
  for (int rr = 0; rr < NR; ++rr)
    for (int off = 32; off > 0; off >>= 1) v[rr] += __shfl_xor(v[rr], off, 64);
  if ((tid & 63) == 0)
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) red[rr * (NT / 64) + (tid >> 6)] = v[rr];
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[rr * (NT / 64) + w];
    v[rr] = t;
  }
}

// The rows are accumulated and stored as TW (double or float; the f and g
// sums in FP64).
// One workgroup per row group; NR = 1: group = one row (rows of all macros
// numbered consecutively by MeshDev::row_off); NR = n_s: group = the n_s
// component rows of one u-node or one trace node (row_off / n_s groups
// before each macro).  Each macro takes the layout of its class.
template <class TW, int NR, int NT>
__global__ void __launch_bounds__(NT) k_form(MeshDev md, FormPtrs fp, TW* __restrict__ Wm) {
  // LDS rows and staged coefficients in the storage type: FP64 for the FP64
  // path; FP32 for the FP32 path (its sums carry no cancellation beyond
  // FP32 rounding, and half the LDS lets two workgroups share a CU)
  using TL = TW;
  extern __shared__ __align__(16) unsigned char form_smem[];
  TL* row = reinterpret_cast<TL*>(form_smem);
  __shared__ double red[NR * (NT / 64)];
  const int tid = threadIdx.x;
  const long long G = fp.group0 + blockIdx.x;
  const int macro = macro_of_row(md.row_off, md.n_macros, G * NR);
  const int g = (int)(G - md.row_off[macro] / NR);
  if (fp.only_class >= 0 && md.macro_class[macro] != fp.only_class) return;
  const ClassDev& cd = class_of(md, macro);
  if (fp.split_cols >= 0 && (NR > 1) != (cd.n_cols <= fp.split_cols)) return;
  const int ns = cd.ns, d = cd.dim, A = cd.A, T = cd.T, N = cd.N;
  const int nsA = fp.nsA, dnsA = fp.dnsA;
  const int n_cols = cd.n_cols, ldr = n_cols;
  TL* sc = row + fp.coef_off;  // staged coefficient rows
  for (int i = tid; i < NR * n_cols; i += NT) row[i] = TL(0);
  // the class's 1D operators, read by every line and face target
  double* C1Ds = reinterpret_cast<double*>(form_smem + fp.tab_off);
  const int tsz = d * cd.nmax1 * cd.nmax1;
  double* Minv1Ds = C1Ds + tsz;
  for (int i = tid; i < tsz; i += NT) {
    C1Ds[i] = cd.C1D[i];
    Minv1Ds[i] = cd.Minv1D[i];
  }
  // rows of the group: r_rr = r0 + rr * rstride
  int r0, rstride;
  bool urow;
  int a = 0, c0 = 0, lf = 0, j = 0, nf = 0;
  if (NR == 1) {
    const int r = g;
    urow = r < cd.n_u;
    if (urow) {
      c0 = r / N; a = r % N;
    } else {
      const int rho = r - cd.n_u;
      while (lf + 1 < 2 * d && rho >= cd.nf_off[lf + 1]) ++lf;
      nf = cd.nf_nodes[lf];
      const int loc = rho - cd.nf_off[lf];
      c0 = loc / nf; j = loc % nf;
    }
    r0 = r; rstride = 0;
    if (fp.duhat && !urow) return;  // uniform per workgroup
  } else {
    urow = g < N;
    if (urow) {
      a = g; c0 = 0;
      r0 = a; rstride = N;
    } else {
      if (fp.duhat) return;  // recovery form: S rows only (uniform per workgroup)
      int rho = g - N;  // trace node index over the local faces
      while (lf + 1 < 2 * d && rho >= cd.nf_nodes[lf]) { rho -= cd.nf_nodes[lf]; ++lf; }
      nf = cd.nf_nodes[lf];
      j = rho; c0 = 0;
      r0 = cd.n_u + cd.nf_off[lf] + j; rstride = nf;
    }
  }
  __syncthreads();
  const double* RQt = fp.RQt + (size_t)d * md.u_off[macro];
  double fpart[NR];
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) fpart[rr] = 0.0;
  if (urow) {
    // ---- u-rows (c0 + rr, a) ----
    const int cnt = cd.node_ne[a];
    for (int ie = 0; ie < cnt; ++ie) {
      const int e = cd.node_e[a * 8 + ie], ae = cd.node_a[a * 8 + ie];
      const long long el = md.el_off[macro] + e;
      // row (c, ae) of the element blocks; component rows are A apart
      const double* auu = fp.AUU + ((size_t)el * nsA + (size_t)(c0 * A + ae)) * nsA;
      const double* auq = fp.AUQ + ((size_t)el * nsA + (size_t)(c0 * A + ae)) * dnsA;
      const size_t su = (size_t)A * nsA, sq = (size_t)A * dnsA;
      const int* en = cd.elem_nodes + (size_t)e * A;
      __syncthreads();
      // the NR rows of A_uq^e, read by every line and face target, go to LDS
      for (int i = tid; i < NR * dnsA; i += NT) {
        const int2 qr = divmod(i, dnsA);
        sc[i] = (TL)auq[qr.x * sq + qr.y];
      }
      for (int i = tid; i < nsA; i += NT) {
        const int2 qr = divmod(i, A);
        const int col = qr.x * N + en[qr.y];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) row[rr * ldr + col] += (TL)auu[rr * su + i];
      }
      __syncthreads();
      // f: A_uq A_qq^{-1} R_Q
      for (int i = tid; i < dnsA; i += NT) {
        const int2 qr = divmod(i, A);
        const int lc = qr.x, b = qr.y;
        const double rq = RQt[(size_t)lc * N + en[b]];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) fpart[rr] += auq[rr * sq + i] * rq;  // FP64 coefficients
      }
      for (int k = 0; k < d; ++k) {
        if (k > 0) __syncthreads();
        auto coef = [&](int rr, int kk, int cp, int b) { return (double)sc[rr * dnsA + (kk * ns + cp) * A + b]; };
        add_direction<NR, NT>(cd, C1Ds, Minv1Ds, e, k, coef, -1.0, 1.0, row, ldr, tid);
      }
      // A_u,uh on the element's macro-boundary faces through node a
      for (int lf2 = 0; lf2 < 2 * d; ++lf2) {
        const int sid = cd.elem_sub[(size_t)e * 2 * d + lf2];
        if (sid < 0) continue;
        const int ta = cd.finv[(size_t)lf2 * A + ae];
        if (ta < 0) continue;
        __syncthreads();
        const double* aub = fp.SUB + ((size_t)md.sub_off[macro] + sid) * fp.sub_stride + fp.off_AUB;
        const int nst = ns * T;
        const int nf2 = cd.nf_nodes[lf2];
        for (int i = tid; i < nst; i += NT) {
          const int2 qr = divmod(i, T);
          const int cp = qr.x, tp = qr.y;
          const int col = cd.n_u + cd.nf_off[lf2] + cp * nf2 + cd.sub_tid[(size_t)sid * T + tp];
#pragma unroll
          for (int rr = 0; rr < NR; ++rr) row[rr * ldr + col] += (TL)aub[(size_t)((c0 + rr) * T + ta) * nst + i];
        }
      }
    }
    block_sum<NR, NT>(fpart, red, tid);
    if (tid == 0)
#pragma unroll
      for (int rr = 0; rr < NR; ++rr)
        row[rr * ldr + n_cols - 1] = (TL)(fpart[rr] - fp.RU[md.u_off[macro] + r0 + rr * rstride]);
  } else {
    // ---- trace rows (lf, c0 + rr, j) ----
    const int tj = cd.tn_base[lf] + j;
    const int nst = ns * T;
    for (int is = 0; is < cd.tn_cnt[tj]; ++is) {
      const int sid = cd.tn_sub[tj * 4 + is], t = cd.tn_t[tj * 4 + is];
      const int e = cd.sub_elem[sid];
      const double* SB = fp.SUB + ((size_t)md.sub_off[macro] + sid) * fp.sub_stride;
      const double* abu = SB + fp.off_ABU + (size_t)(c0 * T + t) * nst;
      const double* abb = SB + fp.off_ABB + (size_t)(c0 * T + t) * nst;
      const double* abq = SB + fp.off_ABQ + (size_t)(c0 * T + t) * (d * nst);
      const size_t sb = (size_t)T * nst, sbq = (size_t)T * d * nst;  // next component row
      const int* en = cd.elem_nodes + (size_t)e * A;
      const int* fn = cd.fnode + lf * T;
      const int* finv = cd.finv + (size_t)lf * A;
      __syncthreads();
      const int dnst = d * nst;
      for (int i = tid; i < NR * dnst; i += NT) {
        const int2 qr = divmod(i, dnst);
        sc[i] = (TL)abq[qr.x * sbq + qr.y];
      }
      for (int i = tid; i < nst; i += NT) {
        const int2 qr = divmod(i, T);
        const int cp = qr.x, tp = qr.y;
        const int cu = cp * N + en[fn[tp]];
        const int cb = cd.n_u + cd.nf_off[lf] + cp * nf + cd.sub_tid[(size_t)sid * T + tp];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
          row[rr * ldr + cu] += (TL)abu[rr * sb + i];
          row[rr * ldr + cb] += (TL)abb[rr * sb + i];
        }
      }
      __syncthreads();
      for (int i = tid; i < d * nst; i += NT) {
        const int2 qr = divmod(i, T);
        const int lc = qr.x, tp = qr.y;
        const double rq = RQt[(size_t)lc * N + en[fn[tp]]];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) fpart[rr] += abq[rr * sbq + i] * rq;  // FP64 coefficients (g)
      }
      for (int k = 0; k < d; ++k) {
        if (k > 0) __syncthreads();
        auto coef = [&](int rr, int kk, int cp, int b) {
          const int tb = finv[b];
          return tb < 0 ? 0.0 : (double)sc[rr * dnst + (kk * ns + cp) * T + tb];
        };
        add_direction<NR, NT>(cd, C1Ds, Minv1Ds, e, k, coef, -1.0, 1.0, row, ldr, tid);
      }
    }
    block_sum<NR, NT>(fpart, red, tid);
    if (tid == 0) {
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) {
        const int rho = r0 + rr * rstride - cd.n_u;
        const double gv = fpart[rr] - fp.RBloc[md.b_off[macro] + rho];
        if (fp.gloc) {
          fp.gloc[md.b_off[macro] + rho] = gv;
          row[rr * ldr + n_cols - 1] = TL(0);
        } else {
          row[rr * ldr + n_cols - 1] = (TL)gv;
        }
      }
    }
  }
  __syncthreads();
  TW* Wmac = Wm + md.w_off[macro];
  if (fp.duhat) {
    // f + C duhat = f - (-C) duhat from the row's trace columns
    double dot[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) dot[rr] = 0.0;
    for (int s = tid; s < cd.n_b; s += NT) {
      int lf2 = 0;
      while (lf2 + 1 < 2 * d && s >= cd.nf_off[lf2 + 1]) ++lf2;
      const int F = md.macro_face[(size_t)macro * 2 * d + lf2];
      const double xv = fp.duhat[md.face_off[F] + (s - cd.nf_off[lf2])];
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) dot[rr] += (double)row[rr * ldr + cd.n_u + s] * xv;
    }
    block_sum<NR, NT>(dot, red, tid);
    __syncthreads();  // every thread has read the trace columns
    if (tid == 0)
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) row[rr * ldr + cd.n_u] = (TL)((double)row[rr * ldr + n_cols - 1] - dot[rr]);
    __syncthreads();
    const int cend = min(cd.ldw, (cd.n_u + 1 + 63) / 64 * 64);
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
      TW* wrow = Wmac + wtix(r0 + rr * rstride, 0, cd.ldw);
      for (int cidx = tid; cidx < cend; cidx += NT)
        wrow[(cidx >> 6) * 1024 + (cidx & 63)] = (cidx <= cd.n_u) ? (TW)row[rr * ldr + cidx] : TW(0);
    }
    return;
  }
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) {
    TW* wrow = Wmac + wtix(r0 + rr * rstride, 0, cd.ldw);  // column c at wrow[(c >> 6) * 1024 + (c & 63)]
    for (int cidx = tid; cidx < cd.ldw; cidx += NT)
      wrow[(cidx >> 6) * 1024 + (cidx & 63)] = (cidx < n_cols) ? (TW)row[rr * ldr + cidx] : TW(0);
  }
}

// Row buffers (n_cols of the largest class taken) and staged coefficient
// rows (A_uq^e rows: d n_s A values; trace rows use d n_s T <= that), then
// (8-byte aligned) the 1D operators C1D and Minv1D of the largest class.
size_t form_tab_off(const HdgContext& c, int nr, size_t elem, int n_cols) {
  return (elem * (size_t)nr * ((size_t)n_cols + (size_t)c.dnsA) + 7) / 8 * 8;
}
size_t form_lds_bytes(const HdgContext& c, int nr, size_t elem, int n_cols) {
  int nm = 1;
  for (const HostClass& k : c.hcs) nm = std::max(nm, k.nmax1);
  return form_tab_off(c, nr, elem, n_cols) + sizeof(double) * 2 * (size_t)c.hm.dim * nm * nm;
}

template <class TW, int NR, int NT>
hipError_t form_launch(HdgContext& c, hipStream_t s, int m0, int m1, TW* W, double* gloc, int only_class, int n_cols,
                       int split_cols, const double* duhat) {
  FormPtrs fp{c.ws.AUU, c.ws.AUQ, c.ws.SUB, c.ws.RU, c.ws.RQt, c.ws.RBloc, gloc,
              c.nsA, c.dnsA, c.sub_stride, c.off_AUB, c.off_ABU, c.off_ABQ, c.off_ABB, c.hm.row_off[m0] / NR,
              NR * n_cols, only_class, split_cols, (int)form_tab_off(c, NR, sizeof(TW), n_cols), duhat};
  const long long nblk = (c.hm.row_off[m1] - c.hm.row_off[m0]) / NR;
  if (nblk <= 0) return hipSuccess;
  const size_t shm = form_lds_bytes(c, NR, sizeof(TW), n_cols);
  hipLaunchKernelGGL((k_form<TW, NR, NT>), dim3((unsigned)nblk), dim3(NT), shm, s, c.md, fp, W);
  return hipGetLastError();
}

template <class TW>
hipError_t form_all(HdgContext& c, hipStream_t s, int m0, int m1, TW* W, double* gloc, int only_class,
                    const double* duhat) {
  // classes whose n_s row buffers fit in LDS go to the grouped launch
  const int ns = c.hm.ns;
  int cols_g = -1, cols_1 = -1;
  for (const HostClass& k : c.hcs) {
    if (form_lds_bytes(c, ns, sizeof(TW), k.n_cols) <= 150 * 1024) cols_g = std::max(cols_g, k.n_cols);
    else cols_1 = std::max(cols_1, k.n_cols);
  }
  const int split = (cols_g >= 0 && cols_1 >= 0) ? cols_g : -1;
  hipError_t e = hipSuccess;
  if (cols_g >= 0)
    e = ns == 5 ? form_launch<TW, 5, 512>(c, s, m0, m1, W, gloc, only_class, cols_g, split, duhat)
                : form_launch<TW, 4, 512>(c, s, m0, m1, W, gloc, only_class, cols_g, split, duhat);
  if (e == hipSuccess && cols_1 >= 0)
    e = form_launch<TW, 1, 256>(c, s, m0, m1, W, gloc, only_class, cols_1, split, duhat);
  return e;
}

}  // namespace

// Groups of n_s rows for the classes whose row buffers fit in LDS (every
// row of a group shares its target indices; 512 threads), single rows of
// 256 threads for the larger classes.
hipError_t launch_form(HdgContext& c, int prec, int m0, int m1, int only_class, const double* rhs_duhat,
                       hipStream_t s) {
  // FP32 storage: g of the trace rows stays in FP64 (it is O(1) per macro but
  // cancels between the two sides of a face in the assembled b-hat)
  double* gloc = prec == 1 ? c.ws.gloc : nullptr;
  if (!s) s = c.stream;
  if (prec == 1)
    return form_all<float>(c, s, m0, m1, reinterpret_cast<float*>(c.ws.Wm), gloc, only_class, rhs_duhat);
  return form_all<double>(c, s, m0, m1, c.ws.Wm, gloc, only_class, rhs_duhat);
}

hipError_t report_progress(HdgContext& c, const char* what, int i, int n) {
  if (!c.progress) return hipSuccess;
  const hipError_t e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) return e;
  std::fprintf(stderr, "[hdg] %s %d of %d done\n", what, i, n);
  std::fflush(stderr);
  return hipSuccess;
}

hipError_t form_stream_ready(HdgContext& c) {
  hipError_t e;
  if (!c.form_stream && (e = hipStreamCreateWithFlags(&c.form_stream, hipStreamNonBlocking)) != hipSuccess) return e;
  for (hipEvent_t& ev : c.form_events)
    if (!ev && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
  return hipSuccess;
}

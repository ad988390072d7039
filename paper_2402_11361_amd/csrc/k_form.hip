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
// One workgroup builds one row; contributions are added element by element
// (and direction by direction) into an LDS row buffer, in a fixed order.
#include "context.h"

namespace {

constexpr int FORM_THREADS = 256;

struct FormPtrs {
  const double *AUU, *AUQ, *SUB, *RU, *RQt, *RBloc;
  double* gloc;  // non-null: g goes here in FP64 and its W entries are 0
  int nsA, dnsA, sub_stride, off_AUB, off_ABU, off_ABQ, off_ABB;
  long long row0;  // first row of the launch (rows of all macros numbered consecutively)
};

__device__ __forceinline__ void digits(int x, int base, int d, int* out) {
  for (int k = 0; k < d; ++k) { out[k] = x % base; x /= base; }
}

// Adds, for direction k, the contributions of one coefficient row
// coef[(k, cp, b)] (element-local nodes b of element e) through
//   line targets  row[cp*N + node(b with b_k -> n_k)] += sgn_line * sum_bk coef * C1D_k[e_k p + b_k][n_k]
//   face targets  row[n_u + nf_off[2k+s] + cp*nf + j(b_tan)] += sgn_face * sign_s * sum_bk coef * Minv_k[e_k p + b_k][end_s]
// mask(b) selects which element nodes carry coefficients (all for u-rows,
// the face nodes of a sub-face for trace rows).
template <class Coef>
__device__ void add_direction(const ClassDev& cd, int e, int k, Coef coef, double sgn_line, double sgn_face,
                              double* row, int tid) {
  const int d = cd.dim, p = cd.p, A1 = p + 1, ns = cd.ns;
  int eidx[3] = {0, 0, 0};
  digits(e, 1, 0, eidx);
  {
    int t = e;
    for (int j = 0; j < d; ++j) { eidx[j] = t % cd.m[j]; t /= cd.m[j]; }
  }
  const int nk = cd.n1[k], nm = cd.nmax1;
  const int T = cd.T;  // (p+1)^(d-1) tangential combinations of an element
  const double* Ck = cd.C1D + (size_t)k * nm * nm;
  const double* Mk = cd.Minv1D + (size_t)k * nm * nm;
  int stride[3] = {1, cd.n1[0], cd.n1[0] * cd.n1[1]};
  // line targets
  for (int i = tid; i < ns * T * nk; i += FORM_THREADS) {
    const int cp = i / (T * nk), r = i % (T * nk), t = r / nk, n = r % nk;
    int td[2] = {0, 0};
    digits(t, A1, d - 1, td);
    int bd[3] = {0, 0, 0}, ti = 0;
    for (int j = 0; j < d; ++j) if (j != k) bd[j] = td[ti++];
    double s = 0.0;
    int node0 = 0;
    for (int j = 0; j < d; ++j) if (j != k) node0 += (eidx[j] * p + bd[j]) * stride[j];
    for (int bk = 0; bk < A1; ++bk) {
      bd[k] = bk;
      const int b = bd[0] + A1 * (bd[1] + A1 * bd[2]);
      const double cv = coef(k, cp, b);
      if (cv != 0.0) s += cv * Ck[(eidx[k] * p + bk) * nm + n];
    }
    if (s != 0.0) row[cp * cd.N + node0 + n * stride[k]] += sgn_line * s;
  }
  // face targets on the two macro faces normal to k
  for (int i = tid; i < 2 * ns * T; i += FORM_THREADS) {
    const int sidx = i / (ns * T), r = i % (ns * T), cp = r / T, t = r % T;
    int td[2] = {0, 0};
    digits(t, A1, d - 1, td);
    int bd[3] = {0, 0, 0}, ti = 0;
    for (int j = 0; j < d; ++j) if (j != k) bd[j] = td[ti++];
    const int end = (sidx == 0) ? 0 : nk - 1;
    const double sgn = (sidx == 0) ? -1.0 : 1.0;
    double s = 0.0;
    for (int bk = 0; bk < A1; ++bk) {
      bd[k] = bk;
      const int b = bd[0] + A1 * (bd[1] + A1 * bd[2]);
      const double cv = coef(k, cp, b);
      if (cv != 0.0) s += cv * Mk[(eidx[k] * p + bk) * nm + end];
    }
    if (s == 0.0) continue;
    // trace node id on face (k, sidx): tangential macro coordinates, lower axis fastest
    int j = 0, mul = 1;
    for (int a = 0; a < d; ++a) {
      if (a == k) continue;
      j += (eidx[a] * p + bd[a]) * mul;
      mul *= cd.n1[a];
    }
    const int lf = 2 * k + sidx;
    row[cd.n_u + cd.nf_off[lf] + cp * cd.nf_nodes[lf] + j] += sgn_face * sgn * s;
  }
}

// The row is accumulated in FP64 and stored as TW (double or float).
// One workgroup per row of all macros' augmented matrices (row offsets
// MeshDev::row_off; each macro takes the layout of its class).
template <class TW>
__global__ void __launch_bounds__(FORM_THREADS) k_form(MeshDev md, FormPtrs fp, TW* __restrict__ Wm) {
  extern __shared__ double row[];
  __shared__ double red[FORM_THREADS];
  const int tid = threadIdx.x;
  const long long gr = fp.row0 + blockIdx.x;
  const int macro = find_in(md.row_off, md.n_macros, gr);
  const int r = (int)(gr - md.row_off[macro]);
  const ClassDev& cd = class_of(md, macro);
  const int ns = cd.ns, d = cd.dim, A = cd.A, T = cd.T, N = cd.N;
  const int nsA = fp.nsA, dnsA = fp.dnsA;
  const int n_cols = cd.n_cols;
  for (int i = tid; i < n_cols; i += FORM_THREADS) row[i] = 0.0;
  __syncthreads();
  const double* RQt = fp.RQt + (size_t)d * md.u_off[macro];
  double fpart = 0.0;
  if (r < cd.n_u) {
    // ---- u-row (c, a) ----
    const int c = r / N, a = r % N;
    const int cnt = cd.node_ne[a];
    for (int ie = 0; ie < cnt; ++ie) {
      const int e = cd.node_e[a * 8 + ie], ae = cd.node_a[a * 8 + ie];
      const long long el = md.el_off[macro] + e;
      const double* auu = fp.AUU + ((size_t)el * nsA + (size_t)(c * A + ae)) * nsA;
      const double* auq = fp.AUQ + ((size_t)el * nsA + (size_t)(c * A + ae)) * dnsA;
      const int* en = cd.elem_nodes + (size_t)e * A;
      __syncthreads();
      for (int i = tid; i < nsA; i += FORM_THREADS) row[(i / A) * N + en[i % A]] += auu[i];
      // f: A_uq A_qq^{-1} R_Q
      for (int i = tid; i < dnsA; i += FORM_THREADS) {
        const int lc = i / A, b = i % A;
        fpart += auq[i] * RQt[(size_t)lc * N + en[b]];
      }
      for (int k = 0; k < d; ++k) {
        __syncthreads();
        auto coef = [&](int kk, int cp, int b) { return auq[(kk * ns + cp) * A + b]; };
        add_direction(cd, e, k, coef, -1.0, 1.0, row, tid);
      }
      // A_u,uh on the element's macro-boundary faces through node a
      for (int lf = 0; lf < 2 * d; ++lf) {
        const int sid = cd.elem_sub[(size_t)e * 2 * d + lf];
        if (sid < 0) continue;
        const int ta = cd.finv[(size_t)lf * A + ae];
        if (ta < 0) continue;
        __syncthreads();
        const double* aub = fp.SUB + ((size_t)md.sub_off[macro] + sid) * fp.sub_stride + fp.off_AUB;
        const int nst = ns * T;
        const int nf = cd.nf_nodes[lf];
        for (int i = tid; i < nst; i += FORM_THREADS) {
          const int cp = i / T, tp = i % T;
          row[cd.n_u + cd.nf_off[lf] + cp * nf + cd.sub_tid[(size_t)sid * T + tp]] += aub[(size_t)(c * T + ta) * nst + i];
        }
      }
    }
    red[tid] = fpart;
    __syncthreads();
    for (int w = FORM_THREADS / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) row[n_cols - 1] = red[0] - fp.RU[md.u_off[macro] + r];
  } else {
    // ---- trace row (lf, c, j) ----
    const int rho = r - cd.n_u;
    int lf = 0;
    while (lf + 1 < 2 * d && rho >= cd.nf_off[lf + 1]) ++lf;
    const int nf = cd.nf_nodes[lf];
    const int loc = rho - cd.nf_off[lf], c = loc / nf, j = loc % nf;
    const int tj = cd.tn_base[lf] + j;
    const int nst = ns * T;
    for (int is = 0; is < cd.tn_cnt[tj]; ++is) {
      const int sid = cd.tn_sub[tj * 4 + is], t = cd.tn_t[tj * 4 + is];
      const int e = cd.sub_elem[sid];
      const double* SB = fp.SUB + ((size_t)md.sub_off[macro] + sid) * fp.sub_stride;
      const double* abu = SB + fp.off_ABU + (size_t)(c * T + t) * nst;
      const double* abb = SB + fp.off_ABB + (size_t)(c * T + t) * nst;
      const double* abq = SB + fp.off_ABQ + (size_t)(c * T + t) * (d * nst);
      const int* en = cd.elem_nodes + (size_t)e * A;
      const int* fn = cd.fnode + lf * T;
      const int* finv = cd.finv + (size_t)lf * A;
      __syncthreads();
      for (int i = tid; i < nst; i += FORM_THREADS) {
        const int cp = i / T, tp = i % T;
        row[cp * N + en[fn[tp]]] += abu[i];
        row[cd.n_u + cd.nf_off[lf] + cp * nf + cd.sub_tid[(size_t)sid * T + tp]] += abb[i];
      }
      for (int i = tid; i < d * nst; i += FORM_THREADS) {
        const int lc = i / T, tp = i % T;
        fpart += abq[i] * RQt[(size_t)lc * N + en[fn[tp]]];
      }
      for (int k = 0; k < d; ++k) {
        __syncthreads();
        auto coef = [&](int kk, int cp, int b) {
          const int tb = finv[b];
          return tb < 0 ? 0.0 : abq[(kk * ns + cp) * T + tb];
        };
        add_direction(cd, e, k, coef, -1.0, 1.0, row, tid);
      }
    }
    red[tid] = fpart;
    __syncthreads();
    for (int w = FORM_THREADS / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) {
      const double g = red[0] - fp.RBloc[md.b_off[macro] + rho];
      if (fp.gloc) {
        fp.gloc[md.b_off[macro] + rho] = g;
        row[n_cols - 1] = 0.0;
      } else {
        row[n_cols - 1] = g;
      }
    }
  }
  __syncthreads();
  TW* Wmac = Wm + md.w_off[macro];
  for (int i = tid; i < cd.ldw; i += FORM_THREADS) Wmac[wtix(r, i, cd.ldw)] = (i < n_cols) ? (TW)row[i] : TW(0);
}

}  // namespace

hipError_t launch_form(HdgContext& c, int prec, int m0, int m1) {
  // FP32 storage: g of the trace rows stays in FP64 (it is O(1) per macro but
  // cancels between the two sides of a face in the assembled b-hat)
  FormPtrs fp{c.ws.AUU, c.ws.AUQ, c.ws.SUB, c.ws.RU, c.ws.RQt, c.ws.RBloc, prec == 1 ? c.ws.gloc : nullptr,
              c.nsA, c.dnsA, c.sub_stride, c.off_AUB, c.off_ABU, c.off_ABQ, c.off_ABB, c.hm.row_off[m0]};
  const long long nblk = c.hm.row_off[m1] - c.hm.row_off[m0];
  if (nblk <= 0) return hipSuccess;
  const size_t shm = (size_t)c.n_cols * sizeof(double);  // largest class
  if (prec == 1)
    hipLaunchKernelGGL(k_form<float>, dim3((unsigned)nblk), dim3(FORM_THREADS), shm, c.stream, c.md, fp,
                       reinterpret_cast<float*>(c.ws.Wm));
  else
    hipLaunchKernelGGL(k_form<double>, dim3((unsigned)nblk), dim3(FORM_THREADS), shm, c.stream, c.md, fp, c.ws.Wm);
  return hipGetLastError();
}

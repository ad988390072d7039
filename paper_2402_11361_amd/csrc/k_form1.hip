// First-layer (standard) static condensation of a macro (paper Sec. 3.2,
// eq. C46/C47): q and u are eliminated together from
//     W1 = [[ A_L, B1, f1 ],      A_L = [[A_qq, A_qu], [A_uq, A_uu]]
//           [ D1,  E1, g1 ]]      B1 = [A_q,uh; A_u,uh],  D1 = [A_uh,q, A_uh,u]
//                                 E1 = A_uh,uh,  f1 = -[R_Q; R_U],  g1 = -R_Uh
// so that eliminating the first n_q + n_u columns (partial pivoting among
// those rows) leaves A-hat^{T_i} = E1 - D1 A_L^{-1} B1 and
// b-hat^{T_i} = g1 - D1 A_L^{-1} f1 in the bottom-right corner: the same
// blocks as the second layer, at the cost of a factorisation of order
// n_q + n_u = (d + 1) n_u instead of n_u.  Used to measure the two layers
// against each other; the recovery stays with the second layer.
//
// The geometric blocks come from the 1D macro operators: with the mass
// M = M_0 (x) M_1 (x) M_2 and B_k[a][b] = int phi_b d_k phi_a,
//   A_{q_k q_k} = M,   A_{q_k u} = B_k = B1D_k (x) M_(others),
//   A_{q_k uh} on face (k, s) = -n_k M_(tangential) at the face's node rows.
#include "context.h"

namespace {

constexpr int F1_THREADS = 256;

struct Form1Ptrs {
  const double *AUU, *AUQ, *SUB, *RU, *RQ, *RBloc;
  int nsA, dnsA, sub_stride, off_AUB, off_ABU, off_ABQ, off_ABB;
  int m0;               // first macro of the launch
  int n_rows1, ldw1;    // rows (n_q + n_u + n_b) and tile width of W1
  long long wstride1;   // doubles per tiled W1
};

__global__ void __launch_bounds__(F1_THREADS) k_form1(MeshDev md, Form1Ptrs fp, double* __restrict__ W1) {
  extern __shared__ double row[];
  const int tid = threadIdx.x;
  const int macro = fp.m0 + (int)(blockIdx.x / fp.n_rows1);
  const int r = (int)(blockIdx.x % fp.n_rows1);
  const ClassDev& cd = class_of(md, macro);
  const int ns = cd.ns, d = cd.dim, A = cd.A, T = cd.T, N = cd.N, nm = cd.nmax1;
  const int nq = cd.n_q, nu = cd.n_u, nsA = fp.nsA, dnsA = fp.dnsA;
  const int n_cols = fp.n_rows1 + 1;
  for (int i = tid; i < n_cols; i += F1_THREADS) row[i] = 0.0;
  __syncthreads();
  const int stride[3] = {1, cd.n1[0], cd.n1[0] * cd.n1[1]};
  if (r < nq) {
    // ---- q-row (k, c, a) ----
    const int k = r / (ns * N), c = (r / N) % ns, a = r % N;
    int ai[3] = {0, 0, 0};
    for (int j = 0; j < d; ++j) ai[j] = (a / stride[j]) % cd.n1[j];
    const double* M1 = cd.M1D;
    const double* B1 = cd.B1D + (size_t)k * nm * nm;
    for (int b = tid; b < N; b += F1_THREADS) {
      double m = 1.0, bk = 1.0;
      for (int j = 0; j < d; ++j) {
        const int bj = (b / stride[j]) % cd.n1[j];
        const double mj = M1[((size_t)j * nm + ai[j]) * nm + bj];
        m *= mj;
        bk *= (j == k) ? B1[(size_t)ai[j] * nm + bj] : mj;
      }
      row[(k * ns + c) * N + b] = m;     // A_qq
      row[nq + c * N + b] = bk;          // A_qu
    }
    for (int s = 0; s < 2; ++s) {       // A_q,uh on the faces normal to k
      if (ai[k] != (s == 0 ? 0 : cd.n1[k] - 1)) continue;
      const int lf = 2 * k + s, nf = cd.nf_nodes[lf];
      const double nk = (s == 0) ? -1.0 : 1.0;
      for (int jt = tid; jt < nf; jt += F1_THREADS) {
        double v = -nk;
        int t = jt;
        for (int j = 0; j < d; ++j) {
          if (j == k) continue;
          const int tj = t % cd.n1[j];
          t /= cd.n1[j];
          v *= M1[((size_t)j * nm + ai[j]) * nm + tj];
        }
        row[nq + nu + cd.nf_off[lf] + c * nf + jt] = v;
      }
    }
    if (tid == 0) row[n_cols - 1] = -fp.RQ[(size_t)d * md.u_off[macro] + r];
  } else if (r < nq + nu) {
    // ---- u-row (c, a) ----
    const int ru = r - nq, c = ru / N, a = ru % N;
    const int cnt = cd.node_ne[a];
    for (int ie = 0; ie < cnt; ++ie) {
      const int e = cd.node_e[a * 8 + ie], ae = cd.node_a[a * 8 + ie];
      const long long el = md.el_off[macro] + e;
      const double* auu = fp.AUU + ((size_t)el * nsA + (size_t)(c * A + ae)) * nsA;
      const double* auq = fp.AUQ + ((size_t)el * nsA + (size_t)(c * A + ae)) * dnsA;
      const int* en = cd.elem_nodes + (size_t)e * A;
      __syncthreads();
      for (int i = tid; i < nsA; i += F1_THREADS) row[nq + (i / A) * N + en[i % A]] += auu[i];
      for (int i = tid; i < dnsA; i += F1_THREADS) row[(i / A) * N + en[i % A]] += auq[i];  // (l, c') blocks
      for (int lf = 0; lf < 2 * d; ++lf) {
        const int sid = cd.elem_sub[(size_t)e * 2 * d + lf];
        if (sid < 0) continue;
        const int ta = cd.finv[(size_t)lf * A + ae];
        if (ta < 0) continue;
        __syncthreads();
        const double* aub = fp.SUB + ((size_t)md.sub_off[macro] + sid) * fp.sub_stride + fp.off_AUB;
        const int nst = ns * T, nf = cd.nf_nodes[lf];
        for (int i = tid; i < nst; i += F1_THREADS) {
          const int cp = i / T, tp = i % T;
          row[nq + nu + cd.nf_off[lf] + cp * nf + cd.sub_tid[(size_t)sid * T + tp]] +=
              aub[(size_t)(c * T + ta) * nst + i];
        }
      }
    }
    if (tid == 0) row[n_cols - 1] = -fp.RU[md.u_off[macro] + ru];
  } else {
    // ---- trace row (lf, c, j) ----
    const int rho = r - nq - nu;
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
      __syncthreads();
      for (int i = tid; i < nst; i += F1_THREADS) {
        const int cp = i / T, tp = i % T;
        row[nq + cp * N + en[fn[tp]]] += abu[i];
        row[nq + nu + cd.nf_off[lf] + cp * nf + cd.sub_tid[(size_t)sid * T + tp]] += abb[i];
      }
      for (int i = tid; i < d * nst; i += F1_THREADS) {
        const int lc = i / T, tp = i % T;  // lc = l ns + c'
        row[lc * N + en[fn[tp]]] += abq[i];
      }
    }
    if (tid == 0) row[n_cols - 1] = -fp.RBloc[md.b_off[macro] + rho];
  }
  __syncthreads();
  double* Wmac = W1 + (size_t)(macro - fp.m0) * fp.wstride1;
  for (int i = tid; i < fp.ldw1; i += F1_THREADS) Wmac[wtix(r, i, fp.ldw1)] = (i < n_cols) ? row[i] : 0.0;
}

// A-hat^{T_i} and b-hat^{T_i} of the eliminated W1 to the compact copies.
__global__ void k_extract1(MeshDev md, int m0, const double* __restrict__ W1, long long wstride1, int ldw1, int n_piv,
                           int bcol, double* __restrict__ Ac, double* __restrict__ bloc) {
  const int macro = m0 + blockIdx.y;
  const ClassDev& cd = class_of(md, macro);
  const int nb = cd.n_b;
  const double* Wm = W1 + (size_t)blockIdx.y * wstride1;
  double* Am = Ac + md.a32_off[macro];
  for (int r = blockIdx.x; r < nb; r += gridDim.x) {
    for (int k = threadIdx.x; k < nb; k += blockDim.x) Am[(size_t)r * nb + k] = Wm[wtix(n_piv + r, n_piv + k, ldw1)];
    if (threadIdx.x == 0) bloc[md.b_off[macro] + r] = Wm[wtix(n_piv + r, bcol, ldw1)];
  }
}

}  // namespace

template <class T>
hipError_t lu_eliminate(hipStream_t s, T* W, int batch, long long mat_stride, int ld, int n_piv, int n_rows,
                        int n_cols, int* ipiv, int ipiv_stride, int* status, T* scratch, LuTune tune,
                        hipStream_t s2, hipEvent_t evA, hipEvent_t evF);

// First-layer condensation of every macro (one macro class, chunked
// workspace): W1 of as many macros as the W buffer holds at a time.
hipError_t launch_condense_first_layer(HdgContext& c, int* status) {
  const HostClass& h = c.hcs[0];
  const int n_piv = h.n_q + h.n_u, n_rows1 = n_piv + h.n_b, n_cols1 = n_rows1 + 1;
  const int ldw1 = (n_cols1 + 63) / 64 * 64;
  const long long wstride1 = (long long)((n_rows1 + 15) / 16 * 16) * ldw1;
  // one W1 row in LDS; the elimination's panel holds at most 12288 pivot rows
  if (sizeof(double) * (size_t)n_cols1 > 150 * 1024 || n_piv > 12 * 1024) return hipErrorNotSupported;
  // W1 matrices, then their pivots, inside the W buffer
  const size_t per = sizeof(double) * (size_t)wstride1 + sizeof(int) * (size_t)n_piv + 256;
  const int batch_max = (int)std::min<size_t>(c.hm.n_macros, c.wm_bytes / per);
  if (batch_max < 1) return hipErrorInvalidValue;
  double* W1 = c.ws.Wm;
  int* ipiv = reinterpret_cast<int*>(W1 + (size_t)batch_max * wstride1);
  Form1Ptrs fp{c.ws.AUU, c.ws.AUQ, c.ws.SUB, c.ws.RU, c.ws.RQ, c.ws.RBloc, c.nsA, c.dnsA, c.sub_stride,
               c.off_AUB, c.off_ABU, c.off_ABQ, c.off_ABB, 0, n_rows1, ldw1, wstride1};
  hipError_t e;
  for (int m0 = 0; m0 < c.hm.n_macros; m0 += batch_max) {
    const int nb = std::min(batch_max, c.hm.n_macros - m0);
    fp.m0 = m0;
    hipLaunchKernelGGL(k_form1, dim3((unsigned)((long long)nb * n_rows1)), dim3(F1_THREADS),
                       sizeof(double) * (size_t)n_cols1, c.stream, c.md, fp, W1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = lu_eliminate<double>(c.stream, W1, nb, wstride1, ldw1, n_piv, n_rows1, n_cols1, ipiv, n_piv, status,
                                  c.ws.Uinv, h.tune[0], nullptr, nullptr, nullptr)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_extract1, dim3((unsigned)std::min(h.n_b, 1024), (unsigned)nb), dim3(256), 0, c.stream, c.md,
                       m0, W1, wstride1, ldw1, n_piv, n_cols1 - 1, c.ws.Ac, c.ws.bloc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Linearisation of the macro-element HDG residuals (paper eq. C38 / C242,
// Newton blocks of eq. C312) on gfx950.
//
// One workgroup per element; the element tables (basis values, weights,
// geometric contraction table, face tables) are the same for every macro
// class and come by value, the macro-level ones through the macro's class.
// Pointwise fluxes and their derivatives come
// from physics.h (forward mode for d/du, exact linearity for d/dq).  Element
// blocks are contractions of the pointwise derivative tensors K[(c,c')][(k,q)]
// with the geometric table Tvol[(k,q)][(a,b)] = -dphi_k(x_q)_a phi(x_q)_b;
// macro-boundary faces add the numerical-flux terms and produce the
// trace-row blocks of their sub-face.  Gathers then assemble node residuals
// without atomics (fixed summation order).
#include "context.h"
#include "physics.h"

namespace {

template <int D, int P>
struct Sz {
  static constexpr int NS = D + 2, A1 = P + 1, NQ = P + 2;
  static constexpr int A = (D == 3) ? A1 * A1 * A1 : A1 * A1;
  static constexpr int Q = (D == 3) ? NQ * NQ * NQ : NQ * NQ;
  static constexpr int T = (D == 3) ? A1 * A1 : A1;
  static constexpr int FQ = (D == 3) ? NQ * NQ : NQ;
  static constexpr int NSA = NS * A;
  static constexpr int DNSA = D * NS * A;
  static constexpr int KR = NS * NS * (1 + D);  // rows of the pointwise tensor
  static constexpr int KC = D * Q;             // columns (k, q)
  static constexpr int NST = NS * T;
};

struct LinPtrs {
  double *Kq, *AUU, *AUQ, *RUe, *RQe, *SUB;
  int sub_stride, off_AUB, off_ABU, off_ABQ, off_ABB, off_RB;
};

constexpr int LIN_THREADS = 256;
constexpr int KCHUNK = 64;

template <int D, int P>
__global__ void __launch_bounds__(LIN_THREADS)
k_lin_elem(ClassDev ce, MeshDev md, PhysDev ph, StageArgs sa, const double* __restrict__ qg,
           const double* __restrict__ ug, const double* __restrict__ uhg, const double* __restrict__ wg, LinPtrs lp) {
  using S_ = Sz<D, P>;
  constexpr int NS = S_::NS, A = S_::A, Q = S_::Q, T = S_::T, FQ = S_::FQ;
  constexpr int NSA = S_::NSA, DNSA = S_::DNSA, KC = S_::KC, NST = S_::NST;
  const int tid = threadIdx.x;
  const long long el = blockIdx.x;
  const int macro = md.elem_macro[el];
  const int e = (int)(el - md.el_off[macro]);
  const ClassDev& cd = class_of(md, macro);
  const bool steady = !(sa.dt < 1e300);
  const double tcoef = steady ? 0.0 : sa.dii / sa.dt;
  const double ptc = (sa.dtau < 1e300) ? 1.0 / sa.dtau : 0.0;

  __shared__ double s_u[NS * A], s_q[D * NS * A], s_w[NS * A];
  __shared__ double s_Wuq[NS * Q], s_Wqq[D * NS * Q], s_Wtt[NS * Q], s_WFG[D * NS * Q];
  __shared__ double s_K[NS * NS * KCHUNK];
  __shared__ int s_nodes[A];
  __shared__ double s_face[FQ * (NS * NS + D * NS * NS + 4 * NS)];
  __shared__ double s_uh[NS * T], s_uD[NS * T];

  const int* en = cd.elem_nodes + (size_t)e * A;
  for (int i = tid; i < A; i += LIN_THREADS) s_nodes[i] = en[i];
  __syncthreads();
  const double* um = ug + md.u_off[macro];
  const double* qm = qg + (size_t)D * md.u_off[macro];
  for (int i = tid; i < NS * A; i += LIN_THREADS) {
    int c = i / A, a = i % A;
    s_u[i] = um[(size_t)c * cd.N + s_nodes[a]];
    s_w[i] = wg ? wg[md.u_off[macro] + (size_t)c * cd.N + s_nodes[a]] : 0.0;
  }
  for (int i = tid; i < D * NS * A; i += LIN_THREADS) {
    int lc = i / A, a = i % A;
    s_q[i] = qm[(size_t)lc * cd.N + s_nodes[a]];
  }
  __syncthreads();

  double* Ke = lp.Kq + (size_t)el * S_::KR * KC;
  // ---- pointwise volume terms ------------------------------------------
  for (int qp = tid; qp < Q; qp += LIN_THREADS) {
    const double* phi = ce.Phi + (size_t)qp * A;
    double uq[NS], qq[D * NS], wq[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c) { uq[c] = 0.0; wq[c] = 0.0; }
#pragma unroll
    for (int i = 0; i < D * NS; ++i) qq[i] = 0.0;
    for (int a = 0; a < A; ++a) {
      const double f = phi[a];
#pragma unroll
      for (int c = 0; c < NS; ++c) { uq[c] += f * s_u[c * A + a]; wq[c] += f * s_w[c * A + a]; }
#pragma unroll
      for (int i = 0; i < D * NS; ++i) qq[i] += f * s_q[i * A + a];
    }
    const double Wq = ce.W[qp];
    double fg[D * NS];
#pragma unroll
    for (int i = 0; i < D * NS; ++i) fg[i] = 0.0;
    ns_flux<D, double>(uq, qq, ph, fg, true, true);
#pragma unroll
    for (int c = 0; c < NS; ++c) {
      s_Wuq[c * Q + qp] = Wq * uq[c];
      s_Wtt[c * Q + qp] = steady ? 0.0 : Wq * (sa.dii * uq[c] + wq[c]) / sa.dt;
    }
#pragma unroll
    for (int i = 0; i < D * NS; ++i) { s_Wqq[i * Q + qp] = Wq * qq[i]; s_WFG[i * Q + qp] = Wq * fg[i]; }
    // d(F+G)/du by forward mode, one direction per pass
    for (int cp = 0; cp < NS; ++cp) {
      Dl ud[NS], qd[D * NS], od[D * NS];
#pragma unroll
      for (int c = 0; c < NS; ++c) ud[c] = Dl{uq[c], c == cp ? 1.0 : 0.0};
#pragma unroll
      for (int i = 0; i < D * NS; ++i) { qd[i] = Dl{qq[i], 0.0}; od[i] = Dl{0.0, 0.0}; }
      ns_flux<D, Dl>(ud, qd, ph, od, true, true);
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NS; ++c) Ke[(size_t)(c * NS + cp) * KC + k * Q + qp] = Wq * od[k * NS + c].d;
    }
    // dG/dq: G is linear in q for fixed u
    for (int l = 0; l < D; ++l)
      for (int cp = 0; cp < NS; ++cp) {
        double qu[D * NS], og[D * NS];
#pragma unroll
        for (int i = 0; i < D * NS; ++i) { qu[i] = 0.0; og[i] = 0.0; }
        qu[l * NS + cp] = 1.0;
        ns_flux<D, double>(uq, qu, ph, og, false, true);
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int c = 0; c < NS; ++c)
            Ke[(size_t)(NS * NS + (l * NS + c) * NS + cp) * KC + k * Q + qp] = Wq * og[k * NS + c];
      }
  }
  __syncthreads();

  // ---- element residual contributions ------------------------------------
  double* RUe = lp.RUe + (size_t)el * NSA;
  double* RQe = lp.RQe + (size_t)el * DNSA;
  for (int i = tid; i < NSA; i += LIN_THREADS) {
    int c = i / A, a = i % A;
    double s = 0.0;
    for (int qp = 0; qp < Q; ++qp) s += ce.Phi[(size_t)qp * A + a] * s_Wtt[c * Q + qp];
    for (int k = 0; k < D; ++k)
      for (int qp = 0; qp < Q; ++qp) s -= ce.dPhi[((size_t)k * Q + qp) * A + a] * s_WFG[(k * NS + c) * Q + qp];
    RUe[i] = s;
  }
  for (int i = tid; i < DNSA; i += LIN_THREADS) {
    int kc = i / A, a = i % A, k = kc / NS, c = kc % NS;
    double s = 0.0;
    for (int qp = 0; qp < Q; ++qp)
      s += ce.Phi[(size_t)qp * A + a] * s_Wqq[kc * Q + qp] + ce.dPhi[((size_t)k * Q + qp) * A + a] * s_Wuq[c * Q + qp];
    RQe[i] = s;
  }

  // ---- element blocks: [25 rows of K] x Tvol, pass 0 = A_uu, pass 1+l = A_uq(l)
  double* AUU = lp.AUU + (size_t)el * NSA * NSA;
  double* AUQ = lp.AUQ + (size_t)el * NSA * DNSA;
  constexpr int NCOL = A * A;
  constexpr int CPT = 2;
  for (int pass = 0; pass <= D; ++pass) {
    for (int cb = 0; cb < NCOL; cb += LIN_THREADS * CPT) {
      double acc[NS * NS][CPT];
#pragma unroll
      for (int r = 0; r < NS * NS; ++r)
#pragma unroll
        for (int j = 0; j < CPT; ++j) acc[r][j] = 0.0;
      for (int k0 = 0; k0 < KC; k0 += KCHUNK) {
        const int kn = min(KCHUNK, KC - k0);
        __syncthreads();
        for (int i = tid; i < NS * NS * kn; i += LIN_THREADS) {
          int r = i / kn, kk = i % kn;
          s_K[r * KCHUNK + kk] = Ke[(size_t)(pass * NS * NS + r) * KC + k0 + kk];
        }
        __syncthreads();
        // unrolled so that the Tvol loads of several k are in flight at once
        // (one wave per SIMD leaves nothing else to hide their latency)
#pragma unroll 4
        for (int kk = 0; kk < kn; ++kk) {
          double t[CPT];
#pragma unroll
          for (int j = 0; j < CPT; ++j) {
            int col = cb + j * LIN_THREADS + tid;
            t[j] = (col < NCOL) ? ce.Tvol[(size_t)(k0 + kk) * NCOL + col] : 0.0;
          }
#pragma unroll
          for (int r = 0; r < NS * NS; ++r) {
            const double kv = s_K[r * KCHUNK + kk];
#pragma unroll
            for (int j = 0; j < CPT; ++j) acc[r][j] += kv * t[j];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        int col = cb + j * LIN_THREADS + tid;
        if (col >= NCOL) continue;
        int a = col / A, b = col % A;
        if (pass == 0) {
          double mass = (tcoef + ptc) * ce.Mel[a * A + b];
#pragma unroll
          for (int c = 0; c < NS; ++c)
#pragma unroll
            for (int cp = 0; cp < NS; ++cp)
              AUU[(size_t)(c * A + a) * NSA + cp * A + b] = acc[c * NS + cp][j] + (c == cp ? mass : 0.0);
        } else {
          const int l = pass - 1;
#pragma unroll
          for (int c = 0; c < NS; ++c)
#pragma unroll
            for (int cp = 0; cp < NS; ++cp)
              AUQ[(size_t)(c * A + a) * DNSA + (l * NS + cp) * A + b] = acc[c * NS + cp][j];
        }
      }
    }
  }
  __syncthreads();

  // ---- macro-boundary faces of this element -------------------------------
  const double svis_m = 1.0 / ph.Re_c, svis_e = 1.0 / (ph.Re_c * (ph.gamma - 1.0) * ph.Pr);
  for (int lf = 0; lf < 2 * D; ++lf) {
    const int sid = cd.elem_sub[(size_t)e * 2 * D + lf];
    if (sid < 0) continue;
    const int kn = lf / 2;
    const double nsgn = (lf % 2 == 0) ? -1.0 : 1.0;
    const int F = md.macro_face[(size_t)macro * 2 * D + lf];
    const int bnd = md.macro_bnd[(size_t)macro * 2 * D + lf];
    const int nf = cd.nf_nodes[lf];
    const int* tidp = cd.sub_tid + (size_t)sid * T;
    const int* fn = ce.fnode + lf * T;
    const double* Psi = ce.Psi + (size_t)lf * FQ * T;
    const double* WF = ce.WF + (size_t)lf * FQ;
    __syncthreads();
    for (int i = tid; i < NS * T; i += LIN_THREADS) {
      int c = i / T, t = i % T;
      size_t gi = (size_t)md.face_off[F] + (size_t)c * nf + tidp[t];
      s_uh[i] = uhg[gi];
      s_uD[i] = (bnd && md.bc_state) ? md.bc_state[gi] : 0.0;
    }
    __syncthreads();
    // pointwise: s_face[f] = {DFU[c][c'] (NS*NS), DFQ[l][c][c'] (D*NS*NS), S[c], fhat[c], uh[c], uD[c]} * WF
    constexpr int FST = NS * NS + D * NS * NS + 4 * NS;
    for (int f = tid; f < FQ; f += LIN_THREADS) {
      double uh[NS], uf[NS], qf[D * NS], uD[NS];
#pragma unroll
      for (int c = 0; c < NS; ++c) { uh[c] = 0.0; uf[c] = 0.0; uD[c] = 0.0; }
#pragma unroll
      for (int i = 0; i < D * NS; ++i) qf[i] = 0.0;
      for (int t = 0; t < T; ++t) {
        const double ps = Psi[f * T + t];
        const int a = fn[t];
#pragma unroll
        for (int c = 0; c < NS; ++c) { uh[c] += ps * s_uh[c * T + t]; uf[c] += ps * s_u[c * A + a]; uD[c] += ps * s_uD[c * T + t]; }
#pragma unroll
        for (int i = 0; i < D * NS; ++i) qf[i] += ps * s_q[i * A + a];
      }
      // frozen lambda_max = |v.n| + c of the trace state
      const double pr = pressure<D>(uh, ph);
      const double cs = sqrt(ph.gamma * pr / uh[0]);
      const double lam = fabs(nsgn * uh[kn + 1] / uh[0]) + cs;
      double Sd[NS];
      Sd[0] = lam;
#pragma unroll
      for (int j = 1; j <= D; ++j) Sd[j] = lam + svis_m;
      Sd[D + 1] = lam + svis_e;
      double fg[D * NS];
#pragma unroll
      for (int i = 0; i < D * NS; ++i) fg[i] = 0.0;
      ns_flux<D, double>(uh, qf, ph, fg, true, true);
      const double wf = WF[f];
      double* sf = s_face + f * FST;
#pragma unroll
      for (int c = 0; c < NS; ++c) {
        sf[NS * NS + D * NS * NS + c] = wf * Sd[c];
        sf[NS * NS + D * NS * NS + NS + c] = wf * (nsgn * fg[kn * NS + c] + Sd[c] * (uf[c] - uh[c]));
        sf[NS * NS + D * NS * NS + 2 * NS + c] = wf * uh[c];
        sf[NS * NS + D * NS * NS + 3 * NS + c] = wf * (uh[c] - uD[c]);
      }
      for (int cp = 0; cp < NS; ++cp) {
        Dl ud[NS], qd[D * NS], od[D * NS];
#pragma unroll
        for (int c = 0; c < NS; ++c) ud[c] = Dl{uh[c], c == cp ? 1.0 : 0.0};
#pragma unroll
        for (int i = 0; i < D * NS; ++i) { qd[i] = Dl{qf[i], 0.0}; od[i] = Dl{0.0, 0.0}; }
        ns_flux<D, Dl>(ud, qd, ph, od, true, true);
#pragma unroll
        for (int c = 0; c < NS; ++c) sf[c * NS + cp] = wf * (nsgn * od[kn * NS + c].d - (c == cp ? Sd[c] : 0.0));
      }
      for (int l = 0; l < D; ++l)
        for (int cp = 0; cp < NS; ++cp) {
          double qu[D * NS], og[D * NS];
#pragma unroll
          for (int i = 0; i < D * NS; ++i) { qu[i] = 0.0; og[i] = 0.0; }
          qu[l * NS + cp] = 1.0;
          ns_flux<D, double>(uh, qu, ph, og, false, true);
#pragma unroll
          for (int c = 0; c < NS; ++c) sf[NS * NS + (l * NS + c) * NS + cp] = wf * nsgn * og[kn * NS + c];
        }
    }
    __syncthreads();
    double* SB = lp.SUB + ((size_t)md.sub_off[macro] + sid) * lp.sub_stride;
    // residual rows
    for (int i = tid; i < NS * T; i += LIN_THREADS) {
      int c = i / T, t = i % T;
      double ru = 0.0, rq = 0.0, rb = 0.0;
      for (int f = 0; f < FQ; ++f) {
        const double ps = Psi[f * T + t];
        const double* sf = s_face + f * FST + NS * NS + D * NS * NS;
        ru += ps * sf[NS + c];
        rq += ps * sf[2 * NS + c];
        rb += ps * (bnd ? sf[3 * NS + c] : sf[NS + c]);
      }
      RUe[c * A + fn[t]] += ru;
      RQe[(kn * NS + c) * A + fn[t]] -= nsgn * rq;
      SB[lp.off_RB + c * T + t] = rb;
    }
    // blocks over (t, t')
    for (int i = tid; i < T * T; i += LIN_THREADS) {
      int t = i / T, tp = i % T;
      double mm[NS], fu[NS * NS], fq[D * NS * NS], m0 = 0.0;
#pragma unroll
      for (int c = 0; c < NS; ++c) mm[c] = 0.0;
#pragma unroll
      for (int j = 0; j < NS * NS; ++j) fu[j] = 0.0;
#pragma unroll
      for (int j = 0; j < D * NS * NS; ++j) fq[j] = 0.0;
      for (int f = 0; f < FQ; ++f) {
        const double pp = Psi[f * T + t] * Psi[f * T + tp];
        const double* sf = s_face + f * FST;
        m0 += pp * WF[f];
#pragma unroll
        for (int c = 0; c < NS; ++c) mm[c] += pp * sf[NS * NS + D * NS * NS + c];
#pragma unroll
        for (int j = 0; j < NS * NS; ++j) fu[j] += pp * sf[j];
#pragma unroll
        for (int j = 0; j < D * NS * NS; ++j) fq[j] += pp * sf[NS * NS + j];
      }
      const int a = fn[t], b = fn[tp];
#pragma unroll
      for (int c = 0; c < NS; ++c) {
        AUU[(size_t)(c * A + a) * NSA + c * A + b] += mm[c];
#pragma unroll
        for (int l = 0; l < D; ++l)
#pragma unroll
          for (int cp = 0; cp < NS; ++cp)
            AUQ[(size_t)(c * A + a) * DNSA + (l * NS + cp) * A + b] += fq[(l * NS + c) * NS + cp];
#pragma unroll
        for (int cp = 0; cp < NS; ++cp) {
          const size_t rc = (size_t)(c * T + t) * NST + cp * T + tp;
          SB[lp.off_AUB + rc] = fu[c * NS + cp];
          SB[lp.off_ABU + rc] = bnd ? 0.0 : (c == cp ? mm[c] : 0.0);
          SB[lp.off_ABB + rc] = bnd ? (c == cp ? m0 : 0.0) : fu[c * NS + cp];
        }
#pragma unroll
        for (int l = 0; l < D; ++l)
#pragma unroll
          for (int cp = 0; cp < NS; ++cp)
            SB[lp.off_ABQ + (size_t)(c * T + t) * (D * NST) + (l * NS + cp) * T + tp] =
                bnd ? 0.0 : fq[(l * NS + c) * NS + cp];
      }
    }
  }
}

// R_U and R_Q node values: sum of the element contributions of the elements
// containing the node, in a fixed order.
// Grid over the nodes of all macros (node offsets u_off / n_s).
__global__ void k_gather_res(MeshDev md, int NSA, int DNSA, const double* __restrict__ RUe,
                             const double* __restrict__ RQe, double* __restrict__ RU, double* __restrict__ RQ,
                             long long total_nodes) {
  const int ns = md.ns, d = md.dim;
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < total_nodes;
       g += (long long)gridDim.x * blockDim.x) {
    // macro of node g: largest i with u_off[i] / ns <= g
    int lo = 0, hi = md.n_macros - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (md.u_off[mid] / ns <= g) lo = mid; else hi = mid - 1;
    }
    const int macro = lo;
    const ClassDev& cd = class_of(md, macro);
    const int N = cd.N, A = cd.A;
    const int n = (int)(g - md.u_off[macro] / ns);
    const int cnt = cd.node_ne[n];
    const long long e0 = md.el_off[macro];
    for (int c = 0; c < ns; ++c) {
      double s = 0.0;
      for (int i = 0; i < cnt; ++i) {
        const long long el = e0 + cd.node_e[n * 8 + i];
        s += RUe[el * NSA + c * A + cd.node_a[n * 8 + i]];
      }
      RU[md.u_off[macro] + (size_t)c * N + n] = s;
    }
    for (int kc = 0; kc < d * ns; ++kc) {
      double s = 0.0;
      for (int i = 0; i < cnt; ++i) {
        const long long el = e0 + cd.node_e[n * 8 + i];
        s += RQe[el * DNSA + kc * A + cd.node_a[n * 8 + i]];
      }
      RQ[(size_t)d * md.u_off[macro] + (size_t)kc * N + n] = s;
    }
  }
}

// Per-macro trace residual R_Uhat^(i): sum over the sub-faces containing each
// trace node.
__global__ void k_gather_rb(MeshDev md, const double* __restrict__ SUB, int sub_stride, int off_RB,
                            double* __restrict__ RBloc) {
  const long long total = md.b_off[md.n_macros];
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < total; g += (long long)gridDim.x * blockDim.x) {
    const int macro = find_in(md.b_off, md.n_macros, g);
    const ClassDev& cd = class_of(md, macro);
    const int T = cd.T;
    int r = (int)(g - md.b_off[macro]);
    int lf = 0;
    while (lf + 1 < 2 * cd.dim && r >= cd.nf_off[lf + 1]) ++lf;
    const int nf = cd.nf_nodes[lf];
    const int loc = r - cd.nf_off[lf];
    const int c = loc / nf, j = loc % nf;
    const int tj = cd.tn_base[lf] + j;
    double s = 0.0;
    for (int i = 0; i < cd.tn_cnt[tj]; ++i) {
      const int sid = cd.tn_sub[tj * 4 + i], t = cd.tn_t[tj * 4 + i];
      s += SUB[((size_t)md.sub_off[macro] + sid) * sub_stride + off_RB + c * T + t];
    }
    RBloc[g] = s;
  }
}

// Global R_Uhat: sum of the (one or two) macro sides of every face.
__global__ void k_face_sum(MeshDev md, const double* __restrict__ loc, double* __restrict__ out) {
  const int d = md.dim;
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < md.n_glob; g += (long long)gridDim.x * blockDim.x) {
    // locate face by binary search on face_off
    int lo = 0, hi = md.n_faces - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) / 2;
      if (md.face_off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const int F = lo;
    const int r = (int)(g - md.face_off[F]);
    double s = 0.0;
    // minus side sees the face as its local face 2k+1, plus side as 2k
    int k = 0;
    {
      // axis from either side's table
      int m = md.face_minus[F] >= 0 ? md.face_minus[F] : md.face_plus[F];
      for (int lf = 0; lf < 2 * d; ++lf)
        if (md.macro_face[(size_t)m * 2 * d + lf] == F) { k = lf / 2; break; }
    }
    if (md.face_minus[F] >= 0) {
      const int m = md.face_minus[F];
      s += loc[md.b_off[m] + class_of(md, m).nf_off[2 * k + 1] + r];
    }
    if (md.face_plus[F] >= 0) {
      const int m = md.face_plus[F];
      s += loc[md.b_off[m] + class_of(md, m).nf_off[2 * k] + r];
    }
    out[g] = s;
  }
}

// RQt[k][c] = M^{-1} R_Q[k][c] with M = M_0 (x) M_1 (x) M_2 (tensor-product
// inverse applied axis by axis).  One workgroup per (macro, field).
__global__ void k_minv_fields(MeshDev md, const double* __restrict__ in, double* __restrict__ out, int nfield) {
  extern __shared__ double sh[];
  const int macro = blockIdx.x / nfield, fld = blockIdx.x % nfield;
  const ClassDev& cd = class_of(md, macro);
  const int N = cd.N, nm = cd.nmax1;
  double* a = sh;
  double* b = sh + N;
  const size_t base = (size_t)md.dim * md.u_off[macro];
  const double* src = in + base + (size_t)fld * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) a[i] = src[i];
  __syncthreads();
  for (int k = 0; k < cd.dim; ++k) {
    const double* Mi = cd.Minv1D + (size_t)k * nm * nm;
    const int nk = cd.n1[k];
    const int stride = (k == 0) ? 1 : (k == 1 ? cd.n1[0] : cd.n1[0] * cd.n1[1]);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const int ik = (i / stride) % nk;
      const int base = i - ik * stride;
      double s = 0.0;
      for (int j = 0; j < nk; ++j) s += Mi[ik * nm + j] * a[base + j * stride];
      b[i] = s;
    }
    __syncthreads();
    double* t = a; a = b; b = t;
  }
  double* dst = out + base + (size_t)fld * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) dst[i] = a[i];
}

// squared norms of three vectors -> partial sums (one per block) -> out
__global__ void k_sqnorm3(const double* __restrict__ a, long long na, const double* __restrict__ b, long long nb,
                          const double* __restrict__ c, long long nc, double* __restrict__ partial) {
  __shared__ double sh[3][256];
  double s[3] = {0.0, 0.0, 0.0};
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < na; i += st) s[0] += a[i] * a[i];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nb; i += st) s[1] += b[i] * b[i];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nc; i += st) s[2] += c[i] * c[i];
  for (int j = 0; j < 3; ++j) sh[j][threadIdx.x] = s[j];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int j = 0; j < 3; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) partial[blockIdx.x * 3 + j] = sh[j][0];
}

__global__ void k_sum_partials3(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int i = 0; i < nblk; ++i) s += partial[i * 3 + threadIdx.x];
    out[threadIdx.x] = sqrt(s);
  }
}

template <int D, int P>
hipError_t lin_dispatch(HdgContext& c, const double* q, const double* u, const double* uhat, const double* w,
                        StageArgs sa) {
  LinPtrs lp{c.ws.Kq, c.ws.AUU, c.ws.AUQ, c.ws.RUe, c.ws.RQe, c.ws.SUB,
             c.sub_stride, c.off_AUB, c.off_ABU, c.off_ABQ, c.off_ABB, c.off_RB};
  const long long nel = c.hm.el_off[c.hm.n_macros];
  hipLaunchKernelGGL((k_lin_elem<D, P>), dim3((unsigned)nel), dim3(LIN_THREADS), 0, c.stream, c.cd, c.md, c.ph, sa,
                     q, u, uhat, w, lp);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_linearize(HdgContext& c, const double* q, const double* u, const double* uhat, const double* w,
                            StageArgs sa) {
  hipError_t e = hipErrorInvalidValue;
  const int D = c.cd.dim, P = c.cd.p;
  if (D == 2 && P == 1) e = lin_dispatch<2, 1>(c, q, u, uhat, w, sa);
  else if (D == 2 && P == 2) e = lin_dispatch<2, 2>(c, q, u, uhat, w, sa);
  else if (D == 2 && P == 3) e = lin_dispatch<2, 3>(c, q, u, uhat, w, sa);
  else if (D == 3 && P == 1) e = lin_dispatch<3, 1>(c, q, u, uhat, w, sa);
  else if (D == 3 && P == 2) e = lin_dispatch<3, 2>(c, q, u, uhat, w, sa);
  else if (D == 3 && P == 3) e = lin_dispatch<3, 3>(c, q, u, uhat, w, sa);
  if (e != hipSuccess) return e;
  if (c.ph.supg && (e = launch_supg(c, q, u, w, sa)) != hipSuccess) return e;
  const int nm = c.hm.n_macros;
  const long long nn = c.n_u_tot / c.cd.ns;
  hipLaunchKernelGGL(k_gather_res, dim3((unsigned)std::min<long long>((nn + 255) / 256, 65535)), dim3(256), 0, c.stream,
                     c.md, c.nsA, c.dnsA, c.ws.RUe, c.ws.RQe, c.ws.RU, c.ws.RQ, nn);
  const long long nb = c.hm.b_off[nm];
  hipLaunchKernelGGL(k_gather_rb, dim3((unsigned)std::min<long long>((nb + 255) / 256, 65535)), dim3(256), 0, c.stream,
                     c.md, c.ws.SUB, c.sub_stride, c.off_RB, c.ws.RBloc);
  hipLaunchKernelGGL(k_face_sum, dim3((unsigned)std::min<long long>((c.md.n_glob + 255) / 256, 65535)), dim3(256), 0,
                     c.stream, c.md, c.ws.RBloc, c.ws.RBglob);
  const int nfield = c.cd.dim * c.cd.ns;
  int nmax = 0;
  for (const HostClass& k : c.hcs) nmax = std::max(nmax, k.N);
  hipLaunchKernelGGL(k_minv_fields, dim3((unsigned)(nm * nfield)), dim3(256), 2 * nmax * sizeof(double), c.stream,
                     c.md, c.ws.RQ, c.ws.RQt, nfield);
  return hipGetLastError();
}

hipError_t launch_norms(HdgContext& c, double* out3) {
  const int nblk = 1024;
  hipLaunchKernelGGL(k_sqnorm3, dim3(nblk), dim3(256), 0, c.stream, c.ws.RQ, c.n_q_tot, c.ws.RU, c.n_u_tot,
                     c.ws.RBglob, c.md.n_glob, c.ws.red);
  hipLaunchKernelGGL(k_sum_partials3, dim3(1), dim3(64), 0, c.stream, c.ws.red, nblk, out3);
  return hipGetLastError();
}

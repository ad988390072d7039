// SUPG term of the momentum/energy residual (paper eq. C38b) and its Newton
// blocks, with the reading used throughout: strong residual in group form
//   R(x_q) = (d_ii u + w)/dt + sum_k d_k (F_k + G_k)^I
// built from the nodal interpolants of the fluxes, test operator A_k d_k w
// with A_k = dF_k/du at the quadrature state, and the scalar
//   tau = ((2 d_ii/dt)^2 + (2 (|v| + c) p / h)^2 + (4 mu p^2 / (Re_c rho h^2))^2)^(-1/2)
// (h the smallest element edge); A_k and tau are frozen in the Jacobian.
//
//   R_U[c,a] += sum_q sum_y L[(c,a)][(q,y)] R_y(x_q),
//   L[(c,a)][(q,y)] = W_q tau_q sum_k d_k phi_a(x_q) (A_k)_{yc}(x_q),
// and, with J_k(b) = d(F+G)_k/du and GQ_k(b) = dG_k/dq at node b,
//   dR_y(x_q)/du_{c',b} = sum_k d_k phi_b(x_q) J_k(b)_{yc'} + (d_ii/dt) phi_b(x_q) delta_{yc'},
//   dR_y(x_q)/dq_{l,c',b} = sum_k d_k phi_b(x_q) GQ_k(b)_{y,(l,c')},
// so the element blocks gain A_uu^e += L Ru and A_uq^e += L Rq: one batched
// product per element (k_supg_prep writes L and [Ru | Rq], k_supg_gemm adds
// the products).
#include "context.h"
#include "physics.h"
#include <algorithm>

namespace {

template <int D, int P>
struct SupgSz {
  static constexpr int NS = D + 2, A1 = P + 1, NQ = P + 2;
  static constexpr int A = (D == 3) ? A1 * A1 * A1 : A1 * A1;
  static constexpr int Q = (D == 3) ? NQ * NQ * NQ : NQ * NQ;
  static constexpr int NSA = NS * A, DNSA = D * NS * A;
  static constexpr int QY = Q * NS;          // inner dimension of the products
  static constexpr int NCOL = NSA + DNSA;    // columns of [Ru | Rq]
  // nodal flux derivatives and W tau A_k: in LDS when they fit, otherwise in
  // a per-element global slot (3D p = 3: 229 KB; 3D p = 2 stays in LDS)
  static constexpr int NJ = A * D * NS * NS, NGQ = A * D * D * NS * NS, NLA = Q * D * NS * NS;
  static constexpr bool BIG = (NJ + NGQ + NLA) * 8 > 120 * 1024;
  static constexpr int GSLOT = BIG ? NJ + NGQ + NLA : 0;
};

constexpr int SUPG_THREADS = 256;

template <int D, int P>
__global__ void __launch_bounds__(SUPG_THREADS)
k_supg_prep(MeshDev md, PhysDev ph, StageArgs sa, const double* __restrict__ qg, const double* __restrict__ ug,
            const double* __restrict__ wg, long long el0, double* __restrict__ RUe, double* __restrict__ Lbuf,
            double* __restrict__ Rbuf, double* __restrict__ Gbuf) {
  using Z = SupgSz<D, P>;
  constexpr int NS = Z::NS, A = Z::A, Q = Z::Q, NSA = Z::NSA, QY = Z::QY, NCOL = Z::NCOL;
  const int tid = threadIdx.x;
  const long long el = el0 + blockIdx.x;
  const int macro = md.elem_macro[el];
  const int e = (int)(el - md.el_off[macro]);
  const ClassDev& cd = class_of(md, macro);
  const bool steady = !(sa.dt < 1e300);
  const double tcoef = steady ? 0.0 : sa.dii / sa.dt;

  __shared__ double s_u[NS * A], s_q[D * NS * A], s_w[NS * A];
  __shared__ double s_NF[A * D * NS];            // nodal F + G: [b][k][y]
  __shared__ double l_J[Z::BIG ? 1 : Z::NJ];     // [b][k][y][c']
  __shared__ double l_GQ[Z::BIG ? 1 : Z::NGQ];   // [b][k][y][l][c']
  __shared__ double l_LA[Z::BIG ? 1 : Z::NLA];   // W tau A_k: [q][k][y][c]
  __shared__ double s_R[Q * NS];                 // strong residual [q][y]
  double* gs = Gbuf + (size_t)blockIdx.x * Z::GSLOT;
  double* s_J = Z::BIG ? gs : l_J;
  double* s_GQ = Z::BIG ? gs + Z::NJ : l_GQ;
  double* s_LA = Z::BIG ? gs + Z::NJ + Z::NGQ : l_LA;
  __shared__ int s_nodes[A];

  const int* en = cd.elem_nodes + (size_t)e * A;
  for (int i = tid; i < A; i += SUPG_THREADS) s_nodes[i] = en[i];
  __syncthreads();
  const double* um = ug + md.u_off[macro];
  const double* qm = qg + (size_t)D * md.u_off[macro];
  for (int i = tid; i < NS * A; i += SUPG_THREADS) {
    const int c = i / A, a = i % A;
    s_u[i] = um[(size_t)c * cd.N + s_nodes[a]];
    s_w[i] = wg ? wg[md.u_off[macro] + (size_t)c * cd.N + s_nodes[a]] : 0.0;
  }
  for (int i = tid; i < D * NS * A; i += SUPG_THREADS) {
    const int lc = i / A, a = i % A;
    s_q[i] = qm[(size_t)lc * cd.N + s_nodes[a]];
  }
  __syncthreads();

  // ---- nodal fluxes and their derivatives --------------------------------
  for (int b = tid; b < A; b += SUPG_THREADS) {
    double ub[NS], qb[D * NS], f[D * NS];
#pragma unroll
    for (int c = 0; c < NS; ++c) ub[c] = s_u[c * A + b];
#pragma unroll
    for (int i = 0; i < D * NS; ++i) { qb[i] = s_q[i * A + b]; f[i] = 0.0; }
    ns_flux<D, double>(ub, qb, ph, f, true, true);
#pragma unroll
    for (int i = 0; i < D * NS; ++i) s_NF[b * D * NS + i] = f[i];
    for (int cp = 0; cp < NS; ++cp) {
      Dl ud[NS], qd[D * NS], od[D * NS];
#pragma unroll
      for (int c = 0; c < NS; ++c) ud[c] = Dl{ub[c], c == cp ? 1.0 : 0.0};
#pragma unroll
      for (int i = 0; i < D * NS; ++i) { qd[i] = Dl{qb[i], 0.0}; od[i] = Dl{0.0, 0.0}; }
      ns_flux<D, Dl>(ud, qd, ph, od, true, true);
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int y = 0; y < NS; ++y) s_J[((b * D + k) * NS + y) * NS + cp] = od[k * NS + y].d;
    }
    for (int l = 0; l < D; ++l)
      for (int cp = 0; cp < NS; ++cp) {
        double qu[D * NS], og[D * NS];
#pragma unroll
        for (int i = 0; i < D * NS; ++i) { qu[i] = 0.0; og[i] = 0.0; }
        qu[l * NS + cp] = 1.0;
        ns_flux<D, double>(ub, qu, ph, og, false, true);  // G is linear in q
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int y = 0; y < NS; ++y) s_GQ[(((b * D + k) * NS + y) * D + l) * NS + cp] = og[k * NS + y];
      }
  }
  __syncthreads();

  // ---- quadrature points: strong residual, frozen W tau A_k -------------
  double hmin = cd.h[0];
  for (int k = 1; k < D; ++k) hmin = fmin(hmin, cd.h[k]);
  for (int qp = tid; qp < Q; qp += SUPG_THREADS) {
    const double* phi = cd.Phi + (size_t)qp * A;
    double uq[NS], wq[NS], Rq[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c) { uq[c] = 0.0; wq[c] = 0.0; Rq[c] = 0.0; }
    for (int a = 0; a < A; ++a) {
      const double f = phi[a];
#pragma unroll
      for (int c = 0; c < NS; ++c) { uq[c] += f * s_u[c * A + a]; wq[c] += f * s_w[c * A + a]; }
    }
    for (int k = 0; k < D; ++k) {
      const double* dphi = cd.dPhi + ((size_t)k * Q + qp) * A;
      for (int b = 0; b < A; ++b) {
        const double g = dphi[b];
#pragma unroll
        for (int y = 0; y < NS; ++y) Rq[y] += g * s_NF[(b * D + k) * NS + y];
      }
    }
    if (!steady) {
#pragma unroll
      for (int y = 0; y < NS; ++y) Rq[y] += (sa.dii * uq[y] + wq[y]) / sa.dt;
    }
#pragma unroll
    for (int y = 0; y < NS; ++y) s_R[qp * NS + y] = Rq[y];
    // tau from the quadrature state
    const double rho = uq[0];
    double vv = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) vv += (uq[j + 1] / rho) * (uq[j + 1] / rho);
    const double pr = pressure<D>(uq, ph);
    const double cs = sqrt(ph.gamma * pr / rho);
    const double t_time = steady ? 0.0 : (2.0 * sa.dii / sa.dt) * (2.0 * sa.dii / sa.dt);
    const double t_adv = (2.0 * (sqrt(vv) + cs) * P / hmin) * (2.0 * (sqrt(vv) + cs) * P / hmin);
    const double tv = 4.0 * ph.mu * P * P / (ph.Re_c * rho * hmin * hmin);
    const double tau = 1.0 / sqrt(t_time + t_adv + tv * tv);
    const double wt = cd.W[qp] * tau;
    // A_k = dF_k/du (inviscid) by forward mode, one direction c per pass
    for (int c = 0; c < NS; ++c) {
      Dl ud[NS], qd[D * NS], od[D * NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) ud[j] = Dl{uq[j], j == c ? 1.0 : 0.0};
#pragma unroll
      for (int i = 0; i < D * NS; ++i) { qd[i] = Dl{0.0, 0.0}; od[i] = Dl{0.0, 0.0}; }
      ns_flux<D, Dl>(ud, qd, ph, od, true, false);
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int y = 0; y < NS; ++y) s_LA[((qp * D + k) * NS + y) * NS + c] = wt * od[k * NS + y].d;
    }
  }
  __syncthreads();

  // ---- residual: R_U[c,a] += sum_q sum_k d_k phi_a sum_y (W tau A_k)_{yc} R_y
  double* ru = RUe + (size_t)el * NSA;
  for (int i = tid; i < NSA; i += SUPG_THREADS) {
    const int c = i / A, a = i % A;
    double s = 0.0;
    for (int qp = 0; qp < Q; ++qp)
      for (int k = 0; k < D; ++k) {
        const double g = cd.dPhi[((size_t)k * Q + qp) * A + a];
        double t = 0.0;
#pragma unroll
        for (int y = 0; y < NS; ++y) t += s_LA[((qp * D + k) * NS + y) * NS + c] * s_R[qp * NS + y];
        s += g * t;
      }
    ru[i] += s;
  }
  // ---- L [(c,a)][(q,y)] and [Ru | Rq] [(q,y)][col] of this element -------
  const long long slot = blockIdx.x;
  double* L = Lbuf + (size_t)slot * NSA * QY;
  for (int i = tid; i < NSA * QY; i += SUPG_THREADS) {
    const int row = i / QY, col = i % QY;
    const int c = row / A, a = row % A, qp = col / NS, y = col % NS;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) s += cd.dPhi[((size_t)k * Q + qp) * A + a] * s_LA[((qp * D + k) * NS + y) * NS + c];
    L[i] = s;
  }
  double* R = Rbuf + (size_t)slot * QY * NCOL;
  for (int i = tid; i < QY * NCOL; i += SUPG_THREADS) {
    const int row = i / NCOL, col = i % NCOL;
    const int qp = row / NS, y = row % NS;
    double s = 0.0;
    if (col < NSA) {
      const int cp = col / A, b = col % A;
#pragma unroll
      for (int k = 0; k < D; ++k) s += cd.dPhi[((size_t)k * Q + qp) * A + b] * s_J[((b * D + k) * NS + y) * NS + cp];
      if (y == cp) s += tcoef * cd.Phi[(size_t)qp * A + b];
    } else {
      const int cc = col - NSA, lc = cc / A, b = cc % A;  // lc = l NS + c'
#pragma unroll
      for (int k = 0; k < D; ++k)
        s += cd.dPhi[((size_t)k * Q + qp) * A + b] * s_GQ[((b * D + k) * NS + y) * D * NS + lc];
    }
    R[i] = s;
  }
}

// C[el] (M x N, leading dimension ldc) += A[el] (M x K, row-major) B[el]
// (K x N, leading dimension ldb); 32 x 32 output tiles, FP64.
constexpr int GT = 32;
__global__ void __launch_bounds__(256) k_supg_gemm(int M, int N, int K, const double* __restrict__ Ab, long long a_el,
                                                   const double* __restrict__ Bb, long long b_el, int ldb,
                                                   double* __restrict__ Cb, long long c_el0, long long c_el, int ldc) {
  __shared__ double sA[GT][GT + 1];
  __shared__ double sB[GT][GT + 1];
  const long long slot = blockIdx.z;
  const double* A = Ab + slot * a_el;
  const double* B = Bb + slot * b_el;
  double* C = Cb + (c_el0 + slot) * c_el;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const int tx = threadIdx.x % GT, ty = threadIdx.x / GT;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += GT) {
    for (int e = threadIdx.x; e < GT * GT; e += 256) {
      const int r = e / GT, c = e % GT;
      sA[r][c] = (i0 + r < M && k0 + c < K) ? A[(size_t)(i0 + r) * K + k0 + c] : 0.0;
      sB[r][c] = (k0 + r < K && j0 + c < N) ? B[(size_t)(k0 + r) * ldb + j0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < GT; ++k) {
      const double b = sB[k][tx];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] += sA[ty + 8 * r][k] * b;
    }
    __syncthreads();
  }
  const int j = j0 + tx;
  if (j >= N) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty + 8 * r;
    if (i < M) C[(size_t)i * ldc + j] += acc[r];
  }
}

template <int D, int P>
hipError_t supg_dispatch(HdgContext& c, const double* q, const double* u, const double* w, StageArgs sa) {
  using Z = SupgSz<D, P>;
  const long long nel = c.hm.el_off[c.hm.n_macros];
  const long long chunk = c.supg_chunk;
  double* Lbuf = c.ws.supg;
  double* Rbuf = Lbuf + (size_t)chunk * Z::NSA * Z::QY;
  double* Gbuf = Rbuf + (size_t)chunk * Z::QY * Z::NCOL;
  for (long long el0 = 0; el0 < nel; el0 += chunk) {
    const long long ne = std::min(chunk, nel - el0);
    hipLaunchKernelGGL((k_supg_prep<D, P>), dim3((unsigned)ne), dim3(SUPG_THREADS), 0, c.stream, c.md, c.ph, sa, q, u,
                       w, el0, c.ws.RUe, Lbuf, Rbuf, Gbuf);
    // A_uu^e += L Ru,  A_uq^e += L Rq
    dim3 g1((Z::NSA + GT - 1) / GT, (Z::NSA + GT - 1) / GT, (unsigned)ne);
    hipLaunchKernelGGL(k_supg_gemm, g1, dim3(256), 0, c.stream, Z::NSA, Z::NSA, Z::QY, Lbuf, (long long)Z::NSA * Z::QY,
                       Rbuf, (long long)Z::QY * Z::NCOL, Z::NCOL, c.ws.AUU, el0, (long long)Z::NSA * Z::NSA, Z::NSA);
    dim3 g2((Z::DNSA + GT - 1) / GT, (Z::NSA + GT - 1) / GT, (unsigned)ne);
    hipLaunchKernelGGL(k_supg_gemm, g2, dim3(256), 0, c.stream, Z::NSA, Z::DNSA, Z::QY, Lbuf,
                       (long long)Z::NSA * Z::QY, Rbuf + Z::NSA, (long long)Z::QY * Z::NCOL, Z::NCOL, c.ws.AUQ, el0,
                       (long long)Z::NSA * Z::DNSA, Z::DNSA);
  }
  return hipGetLastError();
}

}  // namespace

// Scratch doubles per element of the SUPG products (L and [Ru | Rq], plus
// the global slot of the flux derivatives where they do not fit in LDS).
size_t supg_scratch_per_element(int dim, int p) {
  const int ns = dim + 2, A = (dim == 3) ? (p + 1) * (p + 1) * (p + 1) : (p + 1) * (p + 1);
  const int Q = (dim == 3) ? (p + 2) * (p + 2) * (p + 2) : (p + 2) * (p + 2);
  const size_t nsa = (size_t)ns * A, qy = (size_t)Q * ns;
  size_t gslot = 0;
  if (dim == 3 && p == 3) gslot = SupgSz<3, 3>::GSLOT;
  return nsa * qy + qy * (nsa + (size_t)dim * nsa) + gslot;
}

hipError_t launch_supg(HdgContext& c, const double* q, const double* u, const double* w, StageArgs sa) {
  const int D = c.cd.dim, P = c.cd.p;
  if (D == 2 && P == 1) return supg_dispatch<2, 1>(c, q, u, w, sa);
  if (D == 2 && P == 2) return supg_dispatch<2, 2>(c, q, u, w, sa);
  if (D == 2 && P == 3) return supg_dispatch<2, 3>(c, q, u, w, sa);
  if (D == 3 && P == 1) return supg_dispatch<3, 1>(c, q, u, w, sa);
  if (D == 3 && P == 2) return supg_dispatch<3, 2>(c, q, u, w, sa);
  if (D == 3 && P == 3) return supg_dispatch<3, 3>(c, q, u, w, sa);
  return hipErrorInvalidValue;
}

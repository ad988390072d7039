// Host-side set-up of libhdg.so: box mesh and macro skeleton, reference tables
// of the macro shape (GLL nodes, Gauss rule, Lagrange basis, element and face
// tables, 1D macro operators), workspace plan and upload.
//
// Discretisation (paper Sec. 2.2): u and q are C0 Lagrange of degree p inside
// a macro-element (here a box of m_0 x m_1 [x m_2] tensor-product elements),
// the trace u-hat is C0 Lagrange on each macro face.  Nodes are the
// Gauss-Lobatto-Legendre points of every element; integrals use p + 2 Gauss
// points per direction.
#include "context.h"
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

namespace {

// Legendre P_n and its derivative at x by the three-term recurrence.
void legendre(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1; p1 = pk;
  }
  P = p1;
  // derivative from n (x P_n - P_{n-1}) / (x^2 - 1), valid inside (-1, 1)
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

// Gauss-Lobatto-Legendre points: -1, roots of P_p', +1.
std::vector<double> gll(int p) {
  std::vector<double> x(p + 1);
  x[0] = -1.0; x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double xi = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      // f = P_p'(x); f' = P_p''(x) = (2 x P_p' - p (p+1) P_p) / (1 - x^2)
      double P, dP;
      legendre(p, xi, P, dP);
      double d2 = (2.0 * xi * dP - p * (p + 1.0) * P) / (1.0 - xi * xi);
      double step = dP / d2;
      xi -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[i] = xi;
  }
  std::sort(x.begin(), x.end());
  return x;
}

// Gauss-Legendre rule with n points.
void gauss(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0); w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double xi = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double P = 0, dP = 0;
    for (int it = 0; it < 100; ++it) {
      legendre(n, xi, P, dP);
      double step = P / dP;
      xi -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    legendre(n, xi, P, dP);
    x[i] = xi;
    w[i] = 2.0 / ((1.0 - xi * xi) * dP * dP);
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(n), ws(n);
  for (int i = 0; i < n; ++i) { xs[i] = x[idx[i]]; ws[i] = w[idx[i]]; }
  x = xs; w = ws;
}

// Lagrange basis through nodes g: value and derivative of l_j at x.
void lagrange(const std::vector<double>& g, double x, std::vector<double>& v, std::vector<double>& dv) {
  int n = (int)g.size();
  v.assign(n, 0.0); dv.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double den = 1.0, num = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) { den *= g[j] - g[m]; num *= x - g[m]; }
    v[j] = num / den;
    double s = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == j) continue;
      double t = 1.0;
      for (int m = 0; m < n; ++m)
        if (m != j && m != l) t *= x - g[m];
      s += t;
    }
    dv[j] = s / den;
  }
}

// Dense inverse by Gauss-Jordan elimination with partial pivoting (small n).
std::vector<double> invert(std::vector<double> a, int n) {
  std::vector<double> inv(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
    for (int k = 0; k < n; ++k) { std::swap(a[c * n + k], a[piv * n + k]); std::swap(inv[c * n + k], inv[piv * n + k]); }
    double d = a[c * n + c];
    for (int k = 0; k < n; ++k) { a[c * n + k] /= d; inv[c * n + k] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { a[r * n + k] -= f * a[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
    }
  }
  return inv;
}

int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }

}  // namespace

bool build_mesh(const HdgMeshIn& in, HostMesh& hm, std::string& err) {
  if (in.dim != 2 && in.dim != 3) { err = "dim must be 2 or 3"; return false; }
  if (in.p < 1 || in.p > 3) { err = "p must be 1, 2 or 3"; return false; }
  hm.dim = in.dim; hm.ns = in.dim + 2; hm.p = in.p;
  for (int k = 0; k < 3; ++k) { hm.n_elem[k] = 1; hm.n_seg[k] = 1; hm.periodic[k] = 0; hm.lo[k] = 0; hm.hi[k] = 1; hm.h[k] = 1; }
  for (int k = 0; k < in.dim; ++k) {
    if (in.n_elem[k] < 1 || in.n_seg[k] < 1 || !in.seg_len[k]) { err = "bad mesh size"; return false; }
    if (!(in.hi[k] > in.lo[k])) { err = "hi must exceed lo"; return false; }
    hm.n_elem[k] = in.n_elem[k]; hm.n_seg[k] = in.n_seg[k]; hm.periodic[k] = in.periodic[k] ? 1 : 0;
    hm.lo[k] = in.lo[k]; hm.hi[k] = in.hi[k];
    hm.h[k] = (in.hi[k] - in.lo[k]) / in.n_elem[k];
    hm.seg_len[k].assign(in.seg_len[k], in.seg_len[k] + in.n_seg[k]);
    int s = 0;
    hm.seg_start[k].clear();
    for (int i = 0; i < in.n_seg[k]; ++i) {
      if (hm.seg_len[k][i] < 1) { err = "segment lengths must be positive"; return false; }
      hm.seg_start[k].push_back(s);
      s += hm.seg_len[k][i];
    }
    if (s != in.n_elem[k]) { err = "segments must cover the mesh"; return false; }
  }
  const int d = hm.dim;
  hm.n_macros = 1;
  for (int k = 0; k < d; ++k) hm.n_macros *= hm.n_seg[k];
  auto macro_index = [&](const int s[3]) {
    int i = 0;
    for (int k = d - 1; k >= 0; --k) i = i * hm.n_seg[k] + s[k];
    return i;
  };
  hm.macro_face.assign((size_t)hm.n_macros * 2 * d, -1);
  hm.macro_bnd.assign((size_t)hm.n_macros * 2 * d, 0);
  hm.face_axis.clear(); hm.face_minus.clear(); hm.face_plus.clear(); hm.face_ndof.clear();
  hm.face_nodes.clear(); hm.face_grid.clear();
  for (int k = 0; k < d; ++k) {
    int nb = hm.periodic[k] ? hm.n_seg[k] : hm.n_seg[k] + 1;
    int dims[3] = {1, 1, 1};
    for (int j = 0; j < d; ++j) dims[j] = (j == k) ? nb : hm.n_seg[j];
    int total = dims[0] * dims[1] * dims[2];
    for (int flat = 0; flat < total; ++flat) {
      int c[3] = {0, 0, 0}, t = flat;
      for (int j = 0; j < d; ++j) { c[j] = t % dims[j]; t /= dims[j]; }
      int b = c[k], minus = -1, plus = -1;
      int sm[3] = {c[0], c[1], c[2]}, sp[3] = {c[0], c[1], c[2]};
      if (hm.periodic[k]) {
        sm[k] = (b - 1 + hm.n_seg[k]) % hm.n_seg[k]; sp[k] = b;
        minus = macro_index(sm); plus = macro_index(sp);
      } else {
        if (b > 0) { sm[k] = b - 1; minus = macro_index(sm); }
        if (b < hm.n_seg[k]) { sp[k] = b; plus = macro_index(sp); }
      }
      int nn = 1;
      for (int j = 0; j < d; ++j)
        if (j != k) nn *= hm.seg_len[j][c[j]] * hm.p + 1;
      int fid = (int)hm.face_axis.size();
      hm.face_axis.push_back(k); hm.face_minus.push_back(minus); hm.face_plus.push_back(plus);
      hm.face_nodes.push_back(nn); hm.face_ndof.push_back(nn * hm.ns);
      hm.face_grid.push_back({c[0], c[1], c[2]});
      bool bnd = (minus < 0 || plus < 0);
      if (minus >= 0) { hm.macro_face[(size_t)minus * 2 * d + 2 * k + 1] = fid; hm.macro_bnd[(size_t)minus * 2 * d + 2 * k + 1] = bnd; }
      if (plus >= 0) { hm.macro_face[(size_t)plus * 2 * d + 2 * k + 0] = fid; hm.macro_bnd[(size_t)plus * 2 * d + 2 * k + 0] = bnd; }
    }
  }
  hm.n_faces = (int)hm.face_axis.size();
  hm.face_off.assign(hm.n_faces, 0);
  long long off = 0;
  for (int f = 0; f < hm.n_faces; ++f) { hm.face_off[f] = off; off += hm.face_ndof[f]; }
  hm.n_glob = off;
  // macro classes: distinct element counts per axis, numbered in order of first appearance
  hm.class_m.clear();
  hm.macro_class.assign(hm.n_macros, 0);
  for (int i = 0; i < hm.n_macros; ++i) {
    std::array<int, 3> m{1, 1, 1};
    int t = i;
    for (int k = 0; k < d; ++k) { m[k] = hm.seg_len[k][t % hm.n_seg[k]]; t /= hm.n_seg[k]; }
    int cls = -1;
    for (int j = 0; j < (int)hm.class_m.size(); ++j)
      if (hm.class_m[j] == m) { cls = j; break; }
    if (cls < 0) { cls = (int)hm.class_m.size(); hm.class_m.push_back(m); }
    hm.macro_class[i] = cls;
  }
  hm.n_classes = (int)hm.class_m.size();
  return true;
}

// Coarse multilinear functions of the tangential face coordinates (scaled to
// [0, 1] over the macro face) and the discrete L2 projection onto them with
// the composite Gauss-Lobatto rule of the face nodes as inner product.
static void build_coarse(HostClass& hc) {
  const int d = hc.dim, p = hc.p;
  hc.cq = 1 << (d - 1);
  hc.cF = 2 * d * hc.ns * hc.cq;
  hc.cmaxf = 0;
  for (int lf = 0; lf < 2 * d; ++lf) hc.cmaxf = std::max(hc.cmaxf, hc.nf_nodes[lf]);
  const std::vector<double> x = gll(p);
  std::vector<double> w(p + 1);
  for (int a = 0; a <= p; ++a) {  // Lobatto weights 2 / (p (p+1) P_p(x_a)^2)
    double P, dP;
    legendre(p, x[a], P, dP);
    w[a] = 2.0 / (p * (p + 1.0) * P * P);
  }
  auto composite = [&](int m, std::vector<double>& pos, std::vector<double>& wt) {
    pos.assign(m * p + 1, 0.0);
    wt.assign(m * p + 1, 0.0);
    for (int e = 0; e < m; ++e)
      for (int a = 0; a <= p; ++a) {
        pos[e * p + a] = (e + (x[a] + 1.0) / 2.0) / m;
        wt[e * p + a] += w[a] / (2.0 * m);
      }
  };
  const int cq = hc.cq, mf = hc.cmaxf;
  hc.cR.assign((size_t)d * cq * mf, 0.0);
  hc.cPhi.assign((size_t)d * mf * cq, 0.0);
  for (int k = 0; k < d; ++k) {
    int tang[2] = {0, 0}, nt = 0;
    for (int a = 0; a < d; ++a)
      if (a != k) tang[nt++] = a;
    std::vector<double> s, ws, t(1, 0.0), wt(1, 1.0);
    composite(hc.m[tang[0]], s, ws);
    if (d == 3) composite(hc.m[tang[1]], t, wt);
    const int n0 = (int)s.size(), nn = n0 * (int)t.size();
    std::vector<double> phi((size_t)nn * cq), wq(nn);
    for (int j = 0; j < nn; ++j) {
      const double S = s[j % n0], T = t[j / n0];
      wq[j] = ws[j % n0] * wt[j / n0];
      if (d == 2) {
        phi[j * cq + 0] = 1.0 - S; phi[j * cq + 1] = S;
      } else {
        phi[j * cq + 0] = (1.0 - S) * (1.0 - T); phi[j * cq + 1] = S * (1.0 - T);
        phi[j * cq + 2] = (1.0 - S) * T;         phi[j * cq + 3] = S * T;
      }
    }
    std::vector<double> G(cq * cq, 0.0);
    for (int j = 0; j < nn; ++j)
      for (int a = 0; a < cq; ++a)
        for (int b = 0; b < cq; ++b) G[a * cq + b] += phi[j * cq + a] * wq[j] * phi[j * cq + b];
    const std::vector<double> Gi = invert(G, cq);
    for (int a = 0; a < cq; ++a)
      for (int j = 0; j < nn; ++j) {
        double r = 0.0;
        for (int b = 0; b < cq; ++b) r += Gi[a * cq + b] * phi[j * cq + b] * wq[j];
        hc.cR[((size_t)k * cq + a) * mf + j] = r;
      }
    for (int j = 0; j < nn; ++j)
      for (int a = 0; a < cq; ++a) hc.cPhi[((size_t)k * mf + j) * cq + a] = phi[j * cq + a];
  }
}

void build_class(const HostMesh& hm, HostClass& hc, const std::array<int, 3>& m) {
  const int d = hm.dim, p = hm.p, ns = hm.ns;
  hc.dim = d; hc.p = p; hc.ns = ns; hc.nq = p + 2;
  for (int k = 0; k < 3; ++k) { hc.m[k] = 1; hc.n1[k] = 1; hc.h[k] = hm.h[k]; }
  for (int k = 0; k < d; ++k) { hc.m[k] = m[k]; hc.n1[k] = hc.m[k] * p + 1; }
  hc.N = hc.n1[0] * hc.n1[1] * hc.n1[2];
  hc.E = hc.m[0] * hc.m[1] * hc.m[2];
  const int A1 = p + 1, nq = hc.nq;
  hc.A = ipow(A1, d); hc.Q = ipow(nq, d); hc.T = ipow(A1, d - 1); hc.Fq = ipow(nq, d - 1);
  hc.n_u = ns * hc.N; hc.n_q = d * ns * hc.N;
  hc.nmax1 = 1;
  for (int k = 0; k < d; ++k) hc.nmax1 = std::max(hc.nmax1, hc.n1[k]);
  // 1D tables
  std::vector<double> g = gll(p), xq, wq;
  gauss(nq, xq, wq);
  std::vector<double> V1(nq * A1), D1(nq * A1), v, dv;
  for (int i = 0; i < nq; ++i) {
    lagrange(g, xq[i], v, dv);
    for (int a = 0; a < A1; ++a) { V1[i * A1 + a] = v[a]; D1[i * A1 + a] = dv[a]; }
  }
  auto unr = [&](int idx, int base, int* out) { for (int k = 0; k < d; ++k) { out[k] = idx % base; idx /= base; } };
  const int A = hc.A, Q = hc.Q, T = hc.T, Fq = hc.Fq;
  hc.Phi.assign((size_t)Q * A, 1.0); hc.dPhi.assign((size_t)d * Q * A, 1.0); hc.W.assign(Q, 1.0);
  for (int q = 0; q < Q; ++q) {
    int qi[3]; unr(q, nq, qi);
    for (int k = 0; k < d; ++k) hc.W[q] *= wq[qi[k]] * hc.h[k] / 2.0;
    for (int a = 0; a < A; ++a) {
      int ai[3]; unr(a, A1, ai);
      double ph = 1.0;
      for (int k = 0; k < d; ++k) ph *= V1[qi[k] * A1 + ai[k]];
      hc.Phi[(size_t)q * A + a] = ph;
      for (int k = 0; k < d; ++k) {
        double dd = 1.0;
        for (int j = 0; j < d; ++j) dd *= (j == k) ? (2.0 / hc.h[k]) * D1[qi[j] * A1 + ai[j]] : V1[qi[j] * A1 + ai[j]];
        hc.dPhi[((size_t)k * Q + q) * A + a] = dd;
      }
    }
  }
  hc.Tvol.assign((size_t)d * Q * A * A, 0.0);
  for (int k = 0; k < d; ++k)
    for (int q = 0; q < Q; ++q)
      for (int a = 0; a < A; ++a)
        for (int b = 0; b < A; ++b)
          hc.Tvol[((size_t)(k * Q + q)) * A * A + a * A + b] = -hc.dPhi[((size_t)k * Q + q) * A + a] * hc.Phi[(size_t)q * A + b];
  hc.Mel.assign((size_t)A * A, 0.0);
  for (int q = 0; q < Q; ++q)
    for (int a = 0; a < A; ++a)
      for (int b = 0; b < A; ++b) hc.Mel[a * A + b] += hc.W[q] * hc.Phi[(size_t)q * A + a] * hc.Phi[(size_t)q * A + b];
  // face tables
  hc.Psi.assign((size_t)2 * d * Fq * T, 1.0); hc.WF.assign((size_t)2 * d * Fq, 1.0); hc.fnode.assign((size_t)2 * d * T, 0);
  for (int lf = 0; lf < 2 * d; ++lf) {
    int k = lf / 2, s = lf % 2;
    int tang[2] = {-1, -1}, nt = 0;
    for (int j = 0; j < d; ++j) if (j != k) tang[nt++] = j;
    for (int f = 0; f < Fq; ++f) {
      int fi[2] = {0, 0}, t_ = f;
      for (int j = 0; j < d - 1; ++j) { fi[j] = t_ % nq; t_ /= nq; }
      for (int j = 0; j < d - 1; ++j) hc.WF[lf * Fq + f] *= wq[fi[j]] * hc.h[tang[j]] / 2.0;
      for (int t = 0; t < T; ++t) {
        int ti[2] = {0, 0}, tt = t;
        for (int j = 0; j < d - 1; ++j) { ti[j] = tt % A1; tt /= A1; }
        double ps = 1.0;
        for (int j = 0; j < d - 1; ++j) ps *= V1[fi[j] * A1 + ti[j]];
        hc.Psi[((size_t)lf * Fq + f) * T + t] = ps;
      }
    }
    for (int t = 0; t < T; ++t) {
      int ti[2] = {0, 0}, tt = t;
      for (int j = 0; j < d - 1; ++j) { ti[j] = tt % A1; tt /= A1; }
      int ai[3] = {0, 0, 0};
      ai[k] = (s == 0) ? 0 : p;
      for (int j = 0; j < d - 1; ++j) ai[tang[j]] = ti[j];
      hc.fnode[lf * T + t] = ai[0] + A1 * (ai[1] + A1 * ai[2]);
    }
  }
  hc.finv.assign((size_t)2 * d * A, -1);
  for (int lf = 0; lf < 2 * d; ++lf)
    for (int t = 0; t < T; ++t) hc.finv[(size_t)lf * A + hc.fnode[lf * T + t]] = t;
  // macro faces
  int nf_acc = 0;
  for (int lf = 0; lf < 2 * d; ++lf) {
    int k = lf / 2, nn = 1;
    for (int j = 0; j < d; ++j) if (j != k) nn *= hc.n1[j];
    hc.nf_nodes[lf] = nn; hc.nf_off[lf] = nf_acc * ns; nf_acc += nn;
  }
  for (int lf = 2 * d; lf < HDG_MAXF; ++lf) { hc.nf_nodes[lf] = 0; hc.nf_off[lf] = nf_acc * ns; }
  hc.n_b = nf_acc * ns;
  // elements and sub-faces
  const int E = hc.E;
  hc.elem_nodes.assign((size_t)E * A, 0); hc.elem_sub.assign((size_t)E * 2 * d, -1);
  hc.sub_elem.clear(); hc.sub_lf.clear(); hc.sub_tid.clear();
  std::vector<int> eidx((size_t)E * 3, 0);
  for (int e = 0; e < E; ++e) {
    int t_ = e;
    for (int k = 0; k < d; ++k) { eidx[e * 3 + k] = t_ % hc.m[k]; t_ /= hc.m[k]; }
    for (int a = 0; a < A; ++a) {
      int ai[3] = {0, 0, 0}, ta = a;
      for (int k = 0; k < d; ++k) { ai[k] = ta % A1; ta /= A1; }
      int gi[3] = {0, 0, 0};
      for (int k = 0; k < d; ++k) gi[k] = eidx[e * 3 + k] * p + ai[k];
      hc.elem_nodes[(size_t)e * A + a] = gi[0] + hc.n1[0] * (gi[1] + hc.n1[1] * gi[2]);
    }
  }
  for (int lf = 0; lf < 2 * d; ++lf) {
    int k = lf / 2, s = lf % 2;
    int tang[2] = {-1, -1}, nt = 0;
    for (int j = 0; j < d; ++j) if (j != k) tang[nt++] = j;
    for (int e = 0; e < E; ++e) {
      if (eidx[e * 3 + k] != (s == 0 ? 0 : hc.m[k] - 1)) continue;
      int sid = (int)hc.sub_elem.size();
      hc.sub_elem.push_back(e); hc.sub_lf.push_back(lf);
      hc.elem_sub[(size_t)e * 2 * d + lf] = sid;
      for (int t = 0; t < T; ++t) {
        int ti[2] = {0, 0}, tt = t;
        for (int j = 0; j < d - 1; ++j) { ti[j] = tt % A1; tt /= A1; }
        int c0 = eidx[e * 3 + tang[0]] * p + ti[0];
        int id = c0;
        if (d == 3) id += hc.n1[tang[0]] * (eidx[e * 3 + tang[1]] * p + ti[1]);
        hc.sub_tid.push_back(id);
      }
    }
  }
  hc.n_sub = (int)hc.sub_elem.size();
  // node -> element incidence
  hc.node_ne.assign(hc.N, 0); hc.node_e.assign((size_t)hc.N * 8, 0); hc.node_a.assign((size_t)hc.N * 8, 0);
  for (int e = 0; e < E; ++e)
    for (int a = 0; a < A; ++a) {
      int n = hc.elem_nodes[(size_t)e * A + a];
      int c = hc.node_ne[n]++;
      hc.node_e[(size_t)n * 8 + c] = e; hc.node_a[(size_t)n * 8 + c] = a;
    }
  // trace node -> sub-face incidence
  hc.tn_base.assign(2 * d, 0);
  int tot = 0;
  for (int lf = 0; lf < 2 * d; ++lf) { hc.tn_base[lf] = tot; tot += hc.nf_nodes[lf]; }
  hc.tn_cnt.assign(tot, 0); hc.tn_sub.assign((size_t)tot * 4, 0); hc.tn_t.assign((size_t)tot * 4, 0);
  for (int sid = 0; sid < hc.n_sub; ++sid) {
    int lf = hc.sub_lf[sid];
    for (int t = 0; t < T; ++t) {
      int j = hc.tn_base[lf] + hc.sub_tid[(size_t)sid * T + t];
      int c = hc.tn_cnt[j]++;
      hc.tn_sub[(size_t)j * 4 + c] = sid; hc.tn_t[(size_t)j * 4 + c] = t;
    }
  }
  // 1D macro operators per axis: assembled C0 mass M, B[a][b] = int phi_a' phi_b
  const int nm = hc.nmax1;
  hc.C1D.assign((size_t)d * nm * nm, 0.0); hc.Minv1D.assign((size_t)d * nm * nm, 0.0); hc.M1D.assign((size_t)d * nm * nm, 0.0);
  hc.B1D.assign((size_t)d * nm * nm, 0.0);
  for (int k = 0; k < d; ++k) {
    int n = hc.n1[k];
    std::vector<double> M(n * n, 0.0), B(n * n, 0.0);
    for (int e = 0; e < hc.m[k]; ++e)
      for (int i = 0; i < nq; ++i) {
        double w = wq[i] * hc.h[k] / 2.0;
        for (int a = 0; a < A1; ++a)
          for (int b = 0; b < A1; ++b) {
            int ga = e * p + a, gb = e * p + b;
            M[ga * n + gb] += w * V1[i * A1 + a] * V1[i * A1 + b];
            B[ga * n + gb] += w * (2.0 / hc.h[k]) * D1[i * A1 + a] * V1[i * A1 + b];
          }
      }
    std::vector<double> Mi = invert(M, n);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += Mi[a * n + c] * B[c * n + b];
        hc.C1D[((size_t)k * nm + a) * nm + b] = s;
        hc.Minv1D[((size_t)k * nm + a) * nm + b] = Mi[a * n + b];
        hc.M1D[((size_t)k * nm + a) * nm + b] = M[a * n + b];
        hc.B1D[((size_t)k * nm + a) * nm + b] = B[a * n + b];
      }
  }
  build_coarse(hc);
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

void plan_workspace(HdgContext& c) {
  const HostClass& hc = c.hc;  // degree-dependent sizes (the same for every class)
  HostMesh& hm = c.hm;
  const int d = hc.dim, ns = hc.ns, A = hc.A, T = hc.T, Q = hc.Q;
  c.nsA = ns * A; c.dnsA = d * ns * A;
  const int nsT = ns * T;
  c.off_AUB = 0;
  c.off_ABU = c.off_AUB + nsT * nsT;
  c.off_ABQ = c.off_ABU + nsT * nsT;
  c.off_ABB = c.off_ABQ + nsT * d * nsT;
  c.off_RB = c.off_ABB + nsT * nsT;
  c.sub_stride = (int)align_up(c.off_RB + nsT, 4);
  c.Kstride = ns * ns * (1 + d) * d * Q;
  // tiled augmented matrix of every class
  for (HostClass& k : c.hcs) {
    k.n_rows = k.n_u + k.n_b;
    k.n_cols = k.n_u + k.n_b + 1;
    k.ldw = (int)align_up(k.n_cols, 64);
    k.wstride = (long long)align_up(k.n_rows, 16) * k.ldw;
  }
  // per-macro offsets; matrices and pivots grouped by class
  const int nm = hm.n_macros;
  hm.u_off.assign(nm + 1, 0); hm.b_off.assign(nm + 1, 0); hm.el_off.assign(nm + 1, 0);
  hm.sub_off.assign(nm + 1, 0); hm.row_off.assign(nm + 1, 0); hm.a32_off.assign(nm + 1, 0);
  for (int i = 0; i < nm; ++i) {
    const HostClass& k = c.hcs[hm.macro_class[i]];
    hm.u_off[i + 1] = hm.u_off[i] + k.n_u;
    hm.b_off[i + 1] = hm.b_off[i] + k.n_b;
    hm.el_off[i + 1] = hm.el_off[i] + k.E;
    hm.sub_off[i + 1] = hm.sub_off[i] + k.n_sub;
    hm.row_off[i + 1] = hm.row_off[i] + k.n_rows;
    hm.a32_off[i + 1] = hm.a32_off[i] + (long long)k.n_b * k.n_b;
  }
  hm.elem_macro.assign(hm.el_off[nm], 0);
  for (int i = 0; i < nm; ++i)
    for (long long e = hm.el_off[i]; e < hm.el_off[i + 1]; ++e) hm.elem_macro[e] = i;
  const int ncl = hm.n_classes;
  hm.class_count.assign(ncl, 0); hm.class_first.assign(ncl, -1);
  for (int i = 0; i < nm; ++i) {
    const int k = hm.macro_class[i];
    if (hm.class_first[k] < 0) hm.class_first[k] = i;
    ++hm.class_count[k];
  }
  hm.class_w_base.assign(ncl, 0); hm.class_ipiv_base.assign(ncl, 0);
  long long wb = 0, pb = 0;
  for (int k = 0; k < ncl; ++k) {
    hm.class_w_base[k] = wb; hm.class_ipiv_base[k] = pb;
    wb += hm.class_count[k] * c.hcs[k].wstride;
    pb += (long long)hm.class_count[k] * c.hcs[k].n_u;
  }
  // chunks of consecutive macros; inside a chunk's W buffer the matrices are
  // grouped by class (one chunk holding every macro when chunking is off).
  // The first chunk takes the remainder, so that the chunks condensed last,
  // whose eliminations the recovery reuses from W, are full.
  const int per = (hm.chunk_macros > 0 && hm.chunk_macros < nm) ? hm.chunk_macros : nm;
  hm.chunk_first.clear();
  hm.chunk_first.push_back(0);
  for (int i = nm % per; i < nm; i += per)
    if (i > 0) hm.chunk_first.push_back(i);
  hm.chunk_first.push_back(nm);
  const int nch = hm.n_chunks();
  hm.chunk_class_w.assign((size_t)nch * ncl, 0);
  hm.chunk_class_cnt.assign((size_t)nch * ncl, 0);
  hm.chunk_class_rank0.assign((size_t)nch * ncl, 0);
  hm.w_off.assign(nm, 0); hm.ipiv_off.assign(nm, 0);
  std::vector<int> rank(ncl, 0);
  long long w_chunk_max = 0;
  for (int j = 0; j < nch; ++j) {
    int* cnt = &hm.chunk_class_cnt[(size_t)j * ncl];
    for (int i = hm.chunk_first[j]; i < hm.chunk_first[j + 1]; ++i) ++cnt[hm.macro_class[i]];
    long long wb_j = 0;
    for (int k = 0; k < ncl; ++k) {
      hm.chunk_class_w[(size_t)j * ncl + k] = wb_j;
      hm.chunk_class_rank0[(size_t)j * ncl + k] = rank[k];
      wb_j += cnt[k] * c.hcs[k].wstride;
    }
    w_chunk_max = std::max(w_chunk_max, wb_j);
    std::vector<int> r(ncl, 0);
    for (int i = hm.chunk_first[j]; i < hm.chunk_first[j + 1]; ++i) {
      const int k = hm.macro_class[i];
      hm.w_off[i] = hm.chunk_class_w[(size_t)j * ncl + k] + r[k] * c.hcs[k].wstride;
      hm.ipiv_off[i] = hm.class_ipiv_base[k] + (long long)(rank[k] + r[k]) * c.hcs[k].n_u;
      ++r[k];
    }
    for (int k = 0; k < ncl; ++k) rank[k] += cnt[k];
  }
  // factor store: whole leading chunks, never the last chunk of a slot
  // (whose eliminations stay in W)
  hm.store_chunks = 0;
  hm.st_off.assign(nm, -1);
  long long st_elems = 0;
  if (hm.chunked() && hm.store_macros > 0)
    for (int j = 0; j < nch - hm.slots() && hm.chunk_first[j + 1] <= hm.store_macros; ++j) {
      for (int i = hm.chunk_first[j]; i < hm.chunk_first[j + 1]; ++i) {
        const int nu = c.hcs[hm.macro_class[i]].n_u;
        hm.st_off[i] = st_elems;
        st_elems += (long long)((nu + 15) / 16 * 16) * ((nu + 63) / 64 * 64);
      }
      hm.store_chunks = j + 1;
    }
  // slot j % slots of W for chunk j
  const int slots = hm.slots();
  if (slots > 1)
    for (int j = 0; j < nch; ++j) {
      const long long base = (long long)(j % slots) * w_chunk_max;
      for (int k = 0; k < ncl; ++k) hm.chunk_class_w[(size_t)j * ncl + k] += base;
      for (int i = hm.chunk_first[j]; i < hm.chunk_first[j + 1]; ++i) hm.w_off[i] += base;
    }
  const long long n_el = hm.el_off[nm];
  c.n_u_tot = hm.u_off[nm];
  c.n_q_tot = (long long)d * hm.u_off[nm];
  c.n_rows = 0; c.n_cols = 0; c.ldw = 0; c.wstride = 0;
  for (const HostClass& k : c.hcs) {
    c.n_rows = std::max(c.n_rows, k.n_rows); c.n_cols = std::max(c.n_cols, k.n_cols);
    c.ldw = std::max(c.ldw, k.ldw); c.wstride = std::max(c.wstride, k.wstride);
  }
  c.nf_max = 0;
  for (int f = 0; f < hm.n_faces; ++f) c.nf_max = std::max(c.nf_max, hm.face_ndof[f]);
  c.ldf = (int)align_up(2 * c.nf_max, 64);
  // face blocks grouped by size (each group eliminated as one batch)
  {
    std::vector<int> order(hm.n_faces);
    for (int f = 0; f < hm.n_faces; ++f) order[f] = f;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hm.face_ndof[a] < hm.face_ndof[b]; });
    hm.face_slot.assign(hm.n_faces, 0);
    hm.face_groups.clear();
    for (int s = 0; s < hm.n_faces; ++s) {
      const int f = order[s];
      hm.face_slot[f] = s;
      if (hm.face_groups.empty() || hm.face_groups.back()[0] != hm.face_ndof[f])
        hm.face_groups.push_back({hm.face_ndof[f], s, 0});
      ++hm.face_groups.back()[2];
    }
  }
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  struct { size_t Kq, AUU, AUQ, RUe, RQe, SUB, RU, RQ, RQt, RBloc, RBglob, gloc, Wm, ipiv, FW, fpiv, A32, A16, ypart, kry, red, small, Uinv, lrn, kctl, supg, Ac, bloc, Fst; } o;
  const bool chunked = hm.chunked();
  const size_t kq_bytes = sizeof(double) * n_el * c.Kstride;
  // chunked: Kq (used only inside the linearisation) shares the W buffer
  o.Kq = chunked ? 0 : take(kq_bytes);
  o.AUU = take(sizeof(double) * n_el * c.nsA * c.nsA);
  o.AUQ = take(sizeof(double) * n_el * c.nsA * c.dnsA);
  o.RUe = take(sizeof(double) * n_el * c.nsA);
  o.RQe = take(sizeof(double) * n_el * c.dnsA);
  o.SUB = take(sizeof(double) * (size_t)hm.sub_off[nm] * c.sub_stride);
  o.RU = take(sizeof(double) * c.n_u_tot);
  o.RQ = take(sizeof(double) * c.n_q_tot);
  o.RQt = take(sizeof(double) * c.n_q_tot);
  o.RBloc = take(sizeof(double) * (size_t)hm.b_off[nm]);
  o.RBglob = take(sizeof(double) * hm.n_glob);
  o.gloc = take(sizeof(double) * (size_t)hm.b_off[nm]);
  c.fstride = (long long)align_up(2 * c.nf_max, 16) * c.ldf;
  c.wm_bytes = std::max(sizeof(double) * (size_t)w_chunk_max * hm.slots(), chunked ? kq_bytes : 0);
  if (chunked && hm.n_classes == 1) {
    // room for at least one first-layer matrix (order n_q + n_u + n_b) and its pivots
    const HostClass& k = c.hcs[0];
    const size_t rows1 = (size_t)k.n_q + k.n_u + k.n_b, ld1 = (rows1 + 1 + 63) / 64 * 64;
    c.wm_bytes = std::max(c.wm_bytes, sizeof(double) * ((rows1 + 15) / 16 * 16) * ld1 +
                                          sizeof(int) * ((size_t)k.n_q + k.n_u) + 256);
  }
  o.Wm = take(c.wm_bytes);
  if (chunked) o.Kq = o.Wm;
  o.ipiv = take(sizeof(int) * (size_t)c.n_u_tot);
  o.FW = take(sizeof(double) * (size_t)hm.n_faces * c.fstride);
  o.fpiv = take(sizeof(int) * (size_t)hm.n_faces * c.nf_max);
  // FP32 copy of A-hat for the inner solver (not kept when chunked)
  o.A32 = take(chunked ? 0 : sizeof(float) * (size_t)hm.a32_off[nm]);
  o.A16 = take(chunked ? 0 : sizeof(unsigned short) * (size_t)hm.a32_off[nm]);
  o.ypart = take(sizeof(double) * (size_t)hm.b_off[nm]);
  o.kry = take(sizeof(double) * (size_t)(2 * c.kry_restart_max + c.kry_inner_max + 8) * hm.n_glob);
  o.red = take(sizeof(double) * (1 << 20));
  o.small = take(sizeof(double) * 4096);
  // elimination scratch per matrix: a 64 x 64 block inverse, two row permutations,
  // a 128 x 128 unit-lower block inverse and two rounds of tournament candidates
  // (48 sets of 64 rows each) (per class slices when there are several classes)
  o.Uinv = take(sizeof(double) * ((size_t)std::max(hm.n_macros, hm.n_faces) * (64 * 64 + 128 * 128 + 512 + 48 * 64) +
                                  64 * (size_t)hm.n_classes + 64));
  // learned stage: X and Y per macro, the neighbour features (1 + 2d) X,
  // then the BF16 copy of the largest network (neighbour inputs)
  const int lrn_in_max = (1 + 2 * hc.dim) * hc.cF;
  o.lrn = take(sizeof(float) * ((2 + 1 + 2 * (size_t)hc.dim) * (size_t)hm.n_macros * hc.cF + 16) +
               sizeof(unsigned short) * mlp_param_count(lrn_in_max, LRN_MAX_HIDDEN, hc.cF));
  o.kctl = take(sizeof(double) * 8192);
  // SUPG: the per-element products are formed in batches of up to 4096 elements
  // (at most 4096 elements and about 4 GB of products per batch)
  c.supg_chunk = 0;
  if (c.ph.supg) {
    const long long per = (long long)supg_scratch_per_element(hc.dim, hc.p) * (long long)sizeof(double);
    c.supg_chunk = std::max<long long>(1, std::min<long long>({n_el, 4096, (4LL << 30) / per}));
  }
  o.supg = take(sizeof(double) * (size_t)c.supg_chunk * (c.ph.supg ? supg_scratch_per_element(hc.dim, hc.p) : 0));
  o.Ac = take(chunked ? sizeof(double) * (size_t)hm.a32_off[nm] : 0);
  o.bloc = take(chunked ? sizeof(double) * (size_t)hm.b_off[nm] : 0);
  o.Fst = take((hm.store_prec == 1 ? sizeof(float) : sizeof(double)) * (size_t)st_elems);
  c.need_bytes = off;
  // remember offsets in the workspace struct (resolved on bind)
  c.ws.bytes = 0;
  c.ws.Kq = reinterpret_cast<double*>(o.Kq);
  c.ws.AUU = reinterpret_cast<double*>(o.AUU);
  c.ws.AUQ = reinterpret_cast<double*>(o.AUQ);
  c.ws.RUe = reinterpret_cast<double*>(o.RUe);
  c.ws.RQe = reinterpret_cast<double*>(o.RQe);
  c.ws.SUB = reinterpret_cast<double*>(o.SUB);
  c.ws.RU = reinterpret_cast<double*>(o.RU);
  c.ws.RQ = reinterpret_cast<double*>(o.RQ);
  c.ws.RQt = reinterpret_cast<double*>(o.RQt);
  c.ws.RBloc = reinterpret_cast<double*>(o.RBloc);
  c.ws.RBglob = reinterpret_cast<double*>(o.RBglob);
  c.ws.gloc = reinterpret_cast<double*>(o.gloc);
  c.ws.Wm = reinterpret_cast<double*>(o.Wm);
  c.ws.ipiv = reinterpret_cast<int*>(o.ipiv);
  c.ws.FW = reinterpret_cast<double*>(o.FW);
  c.ws.fpiv = reinterpret_cast<int*>(o.fpiv);
  c.ws.A32 = reinterpret_cast<float*>(o.A32);
  c.ws.A16 = reinterpret_cast<unsigned short*>(o.A16);
  c.ws.ypart = reinterpret_cast<double*>(o.ypart);
  c.ws.kry = reinterpret_cast<double*>(o.kry);
  c.ws.red = reinterpret_cast<double*>(o.red);
  c.ws.small = reinterpret_cast<double*>(o.small);
  c.ws.Uinv = reinterpret_cast<double*>(o.Uinv);
  c.ws.lrn = reinterpret_cast<float*>(o.lrn);
  c.ws.kctl = reinterpret_cast<double*>(o.kctl);
  c.ws.supg = reinterpret_cast<double*>(o.supg);
  c.ws.Ac = reinterpret_cast<double*>(o.Ac);
  c.ws.bloc = reinterpret_cast<double*>(o.bloc);
  c.ws.Fst = reinterpret_cast<double*>(o.Fst);
}

void node_coords(const HdgContext& c, double* macro_xyz, double* face_xyz) {
  const HostMesh& hm = c.hm;
  const int d = hm.dim, p = hm.p;
  std::vector<double> g = gll(p);
  auto axis_coord = [&](int k, int seg, int i) {
    int e = i / p, j = i % p;
    if (e == hm.seg_len[k][seg]) { e -= 1; j = p; }
    double x0 = hm.lo[k] + (hm.seg_start[k][seg] + e) * hm.h[k];
    return x0 + hm.h[k] * (g[j] + 1.0) / 2.0;
  };
  if (macro_xyz) {
    size_t o = 0;
    for (int i = 0; i < hm.n_macros; ++i) {
      int s[3] = {0, 0, 0}, t = i;
      for (int k = 0; k < d; ++k) { s[k] = t % hm.n_seg[k]; t /= hm.n_seg[k]; }
      const HostClass& hc = c.hcs[hm.macro_class[i]];
      for (int n = 0; n < hc.N; ++n) {
        int ni[3] = {0, 0, 0}, tn = n;
        for (int k = 0; k < d; ++k) { ni[k] = tn % hc.n1[k]; tn /= hc.n1[k]; }
        for (int k = 0; k < d; ++k) macro_xyz[o++] = axis_coord(k, s[k], ni[k]);
      }
    }
  }
  if (face_xyz) {
    size_t o = 0;
    for (int f = 0; f < hm.n_faces; ++f) {
      int k = hm.face_axis[f];
      const auto& gc = hm.face_grid[f];
      int tang[2] = {-1, -1}, nt = 0;
      for (int j = 0; j < d; ++j) if (j != k) tang[nt++] = j;
      int tn[2] = {1, 1};
      for (int j = 0; j < d - 1; ++j) tn[j] = hm.seg_len[tang[j]][gc[tang[j]]] * p + 1;
      // position along the normal: start of segment b (or the domain end)
      int b = gc[k];
      double xn = (b < hm.n_seg[k]) ? hm.lo[k] + hm.seg_start[k][b] * hm.h[k] : hm.hi[k];
      for (int t1 = 0; t1 < tn[1]; ++t1)
        for (int t0 = 0; t0 < tn[0]; ++t0) {
          double x[3] = {0, 0, 0};
          x[k] = xn;
          x[tang[0]] = axis_coord(tang[0], gc[tang[0]], t0);
          if (d == 3) x[tang[1]] = axis_coord(tang[1], gc[tang[1]], t1);
          for (int j = 0; j < d; ++j) face_xyz[o++] = x[j];
        }
    }
  }
}

template <class Tv>
static const Tv* up(HdgContext& c, const std::vector<Tv>& v) {
  if (v.empty()) return nullptr;
  void* p = nullptr;
  if (hipMalloc(&p, v.size() * sizeof(Tv)) != hipSuccess) throw std::runtime_error("hipMalloc failed for a table");
  c.dev_allocs.push_back(p);
  if (hipMemcpy(p, v.data(), v.size() * sizeof(Tv), hipMemcpyHostToDevice) != hipSuccess)
    throw std::runtime_error("table upload failed");
  return static_cast<const Tv*>(p);
}

static ClassDev upload_class(HdgContext& c, const HostClass& hc) {
  ClassDev cd{};
  cd.dim = hc.dim; cd.p = hc.p; cd.nq = hc.nq; cd.ns = hc.ns;
  for (int k = 0; k < 3; ++k) { cd.m[k] = hc.m[k]; cd.n1[k] = hc.n1[k]; cd.h[k] = hc.h[k]; }
  cd.N = hc.N; cd.E = hc.E; cd.A = hc.A; cd.Q = hc.Q; cd.T = hc.T; cd.Fq = hc.Fq;
  cd.n_u = hc.n_u; cd.n_q = hc.n_q; cd.n_b = hc.n_b; cd.n_sub = hc.n_sub; cd.nmax1 = hc.nmax1;
  for (int i = 0; i < HDG_MAXF; ++i) { cd.nf_nodes[i] = hc.nf_nodes[i]; cd.nf_off[i] = hc.nf_off[i]; }
  cd.Phi = up(c, hc.Phi); cd.dPhi = up(c, hc.dPhi); cd.W = up(c, hc.W); cd.Tvol = up(c, hc.Tvol);
  cd.Mel = up(c, hc.Mel); cd.Psi = up(c, hc.Psi); cd.WF = up(c, hc.WF); cd.fnode = up(c, hc.fnode); cd.finv = up(c, hc.finv);
  cd.elem_nodes = up(c, hc.elem_nodes); cd.elem_sub = up(c, hc.elem_sub); cd.sub_elem = up(c, hc.sub_elem);
  cd.sub_lf = up(c, hc.sub_lf); cd.sub_tid = up(c, hc.sub_tid); cd.node_ne = up(c, hc.node_ne);
  cd.node_e = up(c, hc.node_e); cd.node_a = up(c, hc.node_a); cd.tn_cnt = up(c, hc.tn_cnt);
  cd.tn_sub = up(c, hc.tn_sub); cd.tn_t = up(c, hc.tn_t); cd.tn_base = up(c, hc.tn_base);
  cd.C1D = up(c, hc.C1D); cd.Minv1D = up(c, hc.Minv1D); cd.M1D = up(c, hc.M1D); cd.B1D = up(c, hc.B1D);
  cd.cq = hc.cq; cd.cF = hc.cF; cd.cmaxf = hc.cmaxf;
  cd.cR = up(c, hc.cR); cd.cPhi = up(c, hc.cPhi);
  cd.ldw = hc.ldw; cd.n_rows = hc.n_rows; cd.n_cols = hc.n_cols; cd.wstride = hc.wstride;
  return cd;
}

// Device tables of every class and the mesh (after plan_workspace, which
// fixes the per-class matrix layouts and the per-macro offsets).
void upload_tables(HdgContext& c) {
  c.cds.clear();
  for (const HostClass& hc : c.hcs) c.cds.push_back(upload_class(c, hc));
  c.cd = c.cds[0];
  HostMesh& hm = c.hm;
  MeshDev& md = c.md;
  md.dim = hm.dim; md.ns = hm.ns; md.n_macros = hm.n_macros; md.n_faces = hm.n_faces; md.n_glob = hm.n_glob;
  md.macro_face = up(c, hm.macro_face); md.macro_bnd = up(c, hm.macro_bnd); md.face_off = up(c, hm.face_off);
  md.face_ndof = up(c, hm.face_ndof); md.face_minus = up(c, hm.face_minus); md.face_plus = up(c, hm.face_plus);
  md.cls = up(c, c.cds);
  md.macro_class = up(c, hm.macro_class);
  md.u_off = up(c, hm.u_off); md.b_off = up(c, hm.b_off); md.el_off = up(c, hm.el_off);
  md.elem_macro = up(c, hm.elem_macro); md.sub_off = up(c, hm.sub_off); md.row_off = up(c, hm.row_off);
  md.w_off = up(c, hm.w_off); md.a32_off = up(c, hm.a32_off); md.ipiv_off = up(c, hm.ipiv_off);
  md.face_slot = up(c, hm.face_slot);
  c.st_off_dev = up(c, hm.st_off);
}

// Replaces the device copy of the per-macro W offsets (after a new chunking).
void upload_w_offsets(HdgContext& c) {
  const void* old[2] = {c.md.w_off, c.st_off_dev};
  c.md.w_off = up(c, c.hm.w_off);
  c.st_off_dev = up(c, c.hm.st_off);
  for (const void* o : old)
    for (auto it = c.dev_allocs.begin(); it != c.dev_allocs.end(); ++it)
      if (*it == o) {
        (void)hipFree(*it);
        c.dev_allocs.erase(it);
        break;
      }
}


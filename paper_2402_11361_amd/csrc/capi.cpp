// C ABI of libhdg.so (include/hdg.h): argument checks, workspace binding,
// call sequencing and the Krylov drivers.
//
// Krylov (paper Sec. 4.2): right-preconditioned flexible GMRES(restart) with
// two classical Gram-Schmidt passes; its preconditioner runs `inner_its`
// Arnoldi steps of GMRES (zero start) on the system left-preconditioned by
// the inverse face blocks of A_uh,uh.  The vector work runs in HIP kernels;
// the (restart+1) x restart Hessenberg matrix, its Givens rotations and the
// small least-squares solves stay on the host, one synchronisation per
// Gram-Schmidt pass.
#include "../../include/hdg.h"
#include "context.h"
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <new>
#include <sstream>

hipError_t launch_face_sum(HdgContext& c, const double* base, double* out);
hipError_t launch_zero_ints(hipStream_t s, int* p, int n);

namespace {

void clear_graphs(HdgContext& c) {
  for (auto& kv : c.graphs) (void)hipGraphExecDestroy(kv.second);
  c.graphs.clear();
}

hdg_status fail(HdgContext* c, hdg_status s, const std::string& msg) {
  if (c) c->last_error = msg;
  return s;
}

hdg_status hip_fail(HdgContext* c, hipError_t e, const char* where) {
  return fail(c, HDG_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr)                                  \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return hip_fail(c, _e, #expr); \
  } while (0)

struct Pinned {
  double* p = nullptr;
  size_t n = 0;
};

struct Krylov {
  HdgContext& c;
  long long n;
  double *V, *Z, *Vi, *r, *w, *t, *dev_coef, *partial;
  int restart, inner;
  double* host;  // pinned scratch
  int inner_prec;
  int inner_total = 0;
  bool learned = false;  // add the learned coarse correction in precond()

  // another operator and preconditioner on vectors of length n_op (the nested
  // block skeleton); default: the condensed trace operator of the context
  std::function<hipError_t(const double*, double*)> opA, opM;

  Krylov(HdgContext& cc, int rs, int in, double* hostbuf, int prec, long long n_op = 0)
      : c(cc), restart(rs), inner(in), host(hostbuf), inner_prec(prec) {
    n = n_op > 0 ? n_op : c.md.n_glob;
    double* k = c.ws.kry;
    V = k; k += (size_t)(restart + 1) * n;
    Z = k; k += (size_t)restart * n;
    Vi = k; k += (size_t)(inner + 1) * n;
    r = k; k += n;
    w = k; k += n;
    t = k; k += n;
    dev_coef = c.ws.small + 1024;  // up to 512 doubles (the first 1024 hold the status flags)
    partial = c.ws.red;
  }

  hipError_t dots(int k, const double* Vb, const double* x, double* out_dev) {
    return launch_multidot(c.stream, n, k, Vb, n, x, partial, out_dev);
  }
  hipError_t fetch(const double* dev, int k) {
    hipError_t e = hipMemcpyAsync(host, dev, sizeof(double) * k, hipMemcpyDeviceToHost, c.stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c.stream);
  }
  hipError_t norm(const double* x, double& out) {
    hipError_t e = dots(1, x, x, dev_coef + 448);
    if (e != hipSuccess) return e;
    e = fetch(dev_coef + 448, 1);
    out = std::sqrt(std::max(0.0, host[0]));
    return e;
  }
  // CGS2 of w against rows 0..j of basis B; h (host, j+1 values) = total coefficients
  hipError_t cgs2(const double* B, int j, double* w_, double* h) {
    for (int pass = 0; pass < 2; ++pass) {
      hipError_t e = dots(j + 1, B, w_, dev_coef);
      if (e != hipSuccess) return e;
      e = launch_multiaxpy(c.stream, n, j + 1, B, n, dev_coef, -1.0, w_);
      if (e != hipSuccess) return e;
      e = fetch(dev_coef, j + 1);
      if (e != hipSuccess) return e;
      for (int i = 0; i <= j; ++i) h[i] = (pass == 0 ? 0.0 : h[i]) + host[i];
    }
    return hipSuccess;
  }
  hipError_t apply_A(const double* x, double* y, int prec) { return opA ? opA(x, y) : launch_apply(c, x, y, prec); }
  hipError_t apply_M(const double* x, double* y) { return opM ? opM(x, y) : launch_precond_apply(c, x, y); }

  // ---- device-resident Arnoldi steps (no host synchronisation) -------------
  // control block: H [(restart+1) x restart], cs, sn [restart], g [restart+1],
  // res [restart] (|g_{j+1}| after step j), inner Hessenberg, scalars, dots
  double *dH = nullptr, *dcs = nullptr, *dsn = nullptr, *dg = nullptr, *dres = nullptr, *dHin = nullptr,
         *dsc = nullptr, *dyin = nullptr, *ddot = nullptr;
  void dev_init() {
    double* kc = c.ws.kctl;
    dH = kc; dcs = kc + 4160; dsn = kc + 4224; dg = kc + 4288; dres = kc + 4360;
    dHin = kc + 4432; dsc = kc + 4704; dyin = kc + 4720; ddot = kc + 4800;
  }
  // CGS2 of w against rows 0..j of B; the summed coefficients go to col[i * stride]
  hipError_t cgs2_dev(const double* B, int j, double* w_, double* col, int stride) {
    for (int pass = 0; pass < 2; ++pass) {
      hipError_t e = dots(j + 1, B, w_, ddot);
      if (e != hipSuccess) return e;
      if ((e = launch_multiaxpy(c.stream, n, j + 1, B, n, ddot, -1.0, w_)) != hipSuccess) return e;
      if ((e = launch_accum_col(c.stream, j + 1, ddot, col, stride, pass)) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  // h_out = ||w||, w /= ||w|| (w = 0 stays 0)
  hipError_t normalize_dev(double* w_, double* h_out) {
    hipError_t e = dots(1, w_, w_, dsc + 0);
    if (e != hipSuccess) return e;
    if ((e = launch_norm_finish(c.stream, dsc + 0, h_out, dsc + 2)) != hipSuccess) return e;
    return launch_scale_dev(c.stream, n, dsc + 2, w_, w_);
  }
  hipError_t precond_dev(const double* v, double* z) {
    hipError_t e;
    if (inner <= 0) {
      e = apply_M(v, z);
    } else {
      if ((e = apply_M(v, Vi)) != hipSuccess) return e;
      if ((e = normalize_dev(Vi, dsc + 1)) != hipSuccess) return e;  // beta of the inner solve
      for (int j = 0; j < inner; ++j) {
        double* vn = Vi + (size_t)(j + 1) * n;
        if ((e = apply_A(Vi + (size_t)j * n, t, inner_prec)) != hipSuccess) return e;
        if ((e = apply_M(t, vn)) != hipSuccess) return e;
        if ((e = cgs2_dev(Vi, j, vn, dHin + j, inner)) != hipSuccess) return e;
        if ((e = normalize_dev(vn, dHin + (size_t)(j + 1) * inner + j)) != hipSuccess) return e;
        ++inner_total;
      }
      if ((e = launch_small_ls(c.stream, inner, inner, dHin, dsc + 1, dyin)) != hipSuccess) return e;
      e = launch_lincomb(c.stream, n, inner, Vi, n, dyin, z, 0);
    }
    if (e != hipSuccess || !learned) return e;
    return launch_learned_correction(c, v, z);
  }
  // outer step j of a cycle of length m (Z_j, V_{j+1}, column j of H, Givens)
  hipError_t step_dev(int j, int m) {
    hipError_t e;
    double* wv = V + (size_t)(j + 1) * n;
    if ((e = precond_dev(V + (size_t)j * n, Z + (size_t)j * n)) != hipSuccess) return e;
    if ((e = apply_A(Z + (size_t)j * n, wv, 0)) != hipSuccess) return e;
    if ((e = cgs2_dev(V, j, wv, dH + j, m)) != hipSuccess) return e;
    if ((e = normalize_dev(wv, dH + (size_t)(j + 1) * m + j)) != hipSuccess) return e;
    return launch_givens_step(c.stream, j, m, dH, dcs, dsn, dg, dres);
  }
  // steps [j0, j0 + kk): one captured graph per step (built on first use),
  // launched back to back with no host synchronisation in between
  hipError_t steps_graph(int j0, int kk, int m) {
    for (int j = j0; j < j0 + kk; ++j) {
      hipError_t e = step_graph(j, m);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipError_t step_graph(int j0, int m) {
    const int kk = 1;
    const std::array<int, 8> key{j0, kk, m, inner, inner_prec, c.cond_prec, learned ? 1 : 0, c.have_a32 ? 1 : 0};
    auto it = c.graphs.find(key);
    if (it == c.graphs.end()) {
      hipError_t e;
      if (!c.cap_stream && (e = hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking)) != hipSuccess) return e;
      hipStream_t user = c.stream;
      c.stream = c.cap_stream;
      e = hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal);
      const int tot0 = inner_total;
      for (int j = j0; j < j0 + kk && e == hipSuccess; ++j) e = step_dev(j, m);
      inner_total = tot0;
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(c.cap_stream, &graph);
      c.stream = user;
      if (e == hipSuccess) e = e2;
      hipGraphExec_t exec = nullptr;
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return e;
      it = c.graphs.emplace(key, exec).first;
    }
    inner_total += kk * inner;
    return hipGraphLaunch(it->second, c.stream);
  }

  // z = inner GMRES(inner) on M^{-1} A z = M^{-1} v, zero start (+ learned correction)
  hipError_t precond(const double* v, double* z) {
    hipError_t e = precond_plain(v, z);
    if (e != hipSuccess || !learned) return e;
    return launch_learned_correction(c, v, z);
  }
  hipError_t precond_plain(const double* v, double* z) {
    if (inner <= 0) return apply_M(v, z);
    hipError_t e = apply_M(v, Vi);
    if (e != hipSuccess) return e;
    double beta;
    if ((e = norm(Vi, beta)) != hipSuccess) return e;
    if (beta == 0.0) return launch_scale_copy(c.stream, n, 0.0, v, z);
    if ((e = launch_scale_copy(c.stream, n, 1.0 / beta, Vi, Vi)) != hipSuccess) return e;
    std::vector<double> H((size_t)(inner + 1) * inner, 0.0);
    int k = inner;
    for (int j = 0; j < inner; ++j) {
      if ((e = apply_A(Vi + (size_t)j * n, t, inner_prec)) != hipSuccess) return e;
      if ((e = apply_M(t, Vi + (size_t)(j + 1) * n)) != hipSuccess) return e;
      double h[64];
      if ((e = cgs2(Vi, j, Vi + (size_t)(j + 1) * n, h)) != hipSuccess) return e;
      double hn;
      if ((e = norm(Vi + (size_t)(j + 1) * n, hn)) != hipSuccess) return e;
      for (int i = 0; i <= j; ++i) H[(size_t)i * inner + j] = h[i];
      H[(size_t)(j + 1) * inner + j] = hn;
      ++inner_total;
      if (hn == 0.0) { k = j + 1; break; }
      if ((e = launch_scale_copy(c.stream, n, 1.0 / hn, Vi + (size_t)(j + 1) * n, Vi + (size_t)(j + 1) * n)) != hipSuccess)
        return e;
    }
    // least squares min || beta e1 - H y || by Givens rotations
    std::vector<double> g(k + 1, 0.0), y(k, 0.0), cs(k), sn(k);
    g[0] = beta;
    std::vector<double> R((size_t)(k + 1) * k);
    for (int i = 0; i <= k; ++i)
      for (int j = 0; j < k; ++j) R[(size_t)i * k + j] = H[(size_t)i * inner + j];
    for (int j = 0; j < k; ++j) {
      for (int i = 0; i < j; ++i) {
        double a = R[(size_t)i * k + j], b = R[(size_t)(i + 1) * k + j];
        R[(size_t)i * k + j] = cs[i] * a + sn[i] * b;
        R[(size_t)(i + 1) * k + j] = -sn[i] * a + cs[i] * b;
      }
      double a = R[(size_t)j * k + j], b = R[(size_t)(j + 1) * k + j];
      double rr = std::hypot(a, b);
      cs[j] = rr > 0 ? a / rr : 1.0;
      sn[j] = rr > 0 ? b / rr : 0.0;
      R[(size_t)j * k + j] = rr;
      R[(size_t)(j + 1) * k + j] = 0.0;
      double g0 = g[j];
      g[j] = cs[j] * g0;
      g[j + 1] = -sn[j] * g0;
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int j = i + 1; j < k; ++j) s -= R[(size_t)i * k + j] * y[j];
      y[i] = s / R[(size_t)i * k + i];
    }
    for (int i = 0; i < k; ++i) host[i] = y[i];
    if ((e = hipMemcpyAsync(dev_coef + 256, host, sizeof(double) * k, hipMemcpyHostToDevice, c.stream)) != hipSuccess) return e;
    e = launch_lincomb(c.stream, n, k, Vi, n, dev_coef + 256, z, 0);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c.stream);  // host buffer reused next
  }
};

}  // namespace

struct hdg_ctx_s {
  HdgContext c;
  double* pinned = nullptr;
};

extern "C" {

const char* hdg_status_string(hdg_status s) {
  switch (s) {
    case HDG_OK: return "ok";
    case HDG_EINVAL: return "invalid argument";
    case HDG_ENOMEM: return "workspace missing or too small";
    case HDG_EDEVICE: return "HIP runtime error";
    case HDG_ESINGULAR: return "singular local matrix";
    case HDG_ENOCONV: return "Krylov solver did not converge";
    case HDG_EBREAKDOWN: return "Krylov breakdown";
    case HDG_ENAN: return "non-finite residual";
    case HDG_EUNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

const char* hdg_last_error(hdg_ctx ctx) { return ctx ? ctx->c.last_error.c_str() : "null context"; }

hdg_status hdg_setup_mesh(const hdg_mesh_desc* mesh, const hdg_phys* phys, void* hip_stream, hdg_ctx* out) {
  if (!mesh || !phys || !out) return HDG_EINVAL;
  *out = nullptr;
  hdg_ctx h = new (std::nothrow) hdg_ctx_s();
  if (!h) return HDG_ENOMEM;
  HdgContext& c = h->c;
  HdgMeshIn in{};
  in.dim = mesh->dim;
  in.p = mesh->p;
  for (int k = 0; k < 3; ++k) {
    in.n_elem[k] = mesh->n_elem[k]; in.lo[k] = mesh->lo[k]; in.hi[k] = mesh->hi[k];
    in.periodic[k] = mesh->periodic[k]; in.n_seg[k] = mesh->n_seg[k]; in.seg_len[k] = mesh->seg_len[k];
  }
  std::string err;
  if (!build_mesh(in, c.hm, err)) { delete h; return HDG_EINVAL; }
  if (!(phys->gamma > 1.0) || !(phys->Pr > 0) || !(phys->Re > 0) || !(phys->Mach > 0)) { delete h; return HDG_EINVAL; }
  bool any_bnd = false;
  for (int v : c.hm.macro_bnd) any_bnd |= (v != 0);
  if (any_bnd && !phys->bc_state_host) { delete h; return HDG_EINVAL; }
  c.stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c.device) != hipSuccess || diag_scratch_setup(c.device) != hipSuccess) { delete h; return HDG_EDEVICE; }
  c.hcs.resize(c.hm.n_classes);
  for (int k = 0; k < c.hm.n_classes; ++k) build_class(c.hm, c.hcs[k], c.hm.class_m[k]);
  c.hc = c.hcs[0];
  c.ph.gamma = phys->gamma; c.ph.Pr = phys->Pr; c.ph.Re = phys->Re; c.ph.Mach = phys->Mach; c.ph.mu = 1.0;
  c.ph.Re_c = phys->Re / phys->Mach;
  c.ph.kappa = c.ph.mu / (c.ph.Re_c * c.ph.Pr * (c.ph.gamma - 1.0));
  c.ph.supg = phys->supg;
  plan_workspace(c);
  try {
    upload_tables(c);
    if (any_bnd) {
      std::vector<double> bc(phys->bc_state_host, phys->bc_state_host + c.hm.n_glob);
      void* p = nullptr;
      if (hipMalloc(&p, bc.size() * sizeof(double)) != hipSuccess) throw std::runtime_error("hipMalloc bc");
      c.dev_allocs.push_back(p);
      if (hipMemcpy(p, bc.data(), bc.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        throw std::runtime_error("bc upload");
      c.md.bc_state = static_cast<const double*>(p);
    } else {
      c.md.bc_state = nullptr;
    }
  } catch (const std::exception& ex) {
    for (void* p : c.dev_allocs) (void)hipFree(p);
    delete h;
    return HDG_EDEVICE;
  }
  if (hipHostMalloc((void**)&h->pinned, 8192 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    for (void* p : c.dev_allocs) (void)hipFree(p);
    delete h;
    return HDG_EDEVICE;
  }
  *out = h;
  return HDG_OK;
}

hdg_status hdg_query_sizes(hdg_ctx ctx, hdg_sizes* out) {
  if (!ctx || !out) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  out->n_macros = c.hm.n_macros;
  out->n_glob = c.hm.n_glob;
  out->n_u_tot = c.n_u_tot;
  out->n_q_tot = c.n_q_tot;
  out->n_u_macro = 0;
  out->n_b_macro = 0;
  for (const HostClass& k : c.hcs) {
    out->n_u_macro = std::max(out->n_u_macro, (size_t)k.n_u);
    out->n_b_macro = std::max(out->n_b_macro, (size_t)k.n_b);
  }
  out->workspace_bytes = c.need_bytes;
  out->n_faces = c.hm.n_faces;
  return HDG_OK;
}

hdg_status hdg_macro_offsets(hdg_ctx ctx, long long* u_off, long long* b_off) {
  if (!ctx) return HDG_EINVAL;
  const HostMesh& hm = ctx->c.hm;
  for (int i = 0; i <= hm.n_macros; ++i) {
    if (u_off) u_off[i] = hm.u_off[i];
    if (b_off) b_off[i] = hm.b_off[i];
  }
  return HDG_OK;
}

hdg_status hdg_face_offsets(hdg_ctx ctx, long long* face_off) {
  if (!ctx || !face_off) return HDG_EINVAL;
  const HostMesh& hm = ctx->c.hm;
  for (int f = 0; f < hm.n_faces; ++f) face_off[f] = hm.face_off[f];
  face_off[hm.n_faces] = hm.n_glob;
  return HDG_OK;
}

hdg_status hdg_node_coords(hdg_ctx ctx, double* macro_xyz, double* face_xyz) {
  if (!ctx) return HDG_EINVAL;
  node_coords(ctx->c, macro_xyz, face_xyz);
  return HDG_OK;
}

// Precision code of the inner operator (0 the condensed blocks, 1 FP32
// copy, 2 BF16 copy), making the copy on first use after a condensation.
static hdg_status inner_operator(HdgContext& c, int inner_prec, int* code) {
  if (inner_prec != HDG_FP64 && inner_prec != HDG_FP32 && inner_prec != HDG_BF16)
    return fail(&c, HDG_EINVAL, "bad inner precision");
  if (inner_prec == HDG_FP32 && c.cond_prec == 0 && c.hm.chunked())
    return fail(&c, HDG_EUNSUPPORTED, "FP32 inner operator with chunked FP64 condensation (condense in FP32 instead)");
  if (inner_prec == HDG_BF16 && c.hm.chunked())
    return fail(&c, HDG_EUNSUPPORTED, "BF16 inner operator with chunked condensation");
  if (inner_prec == HDG_FP32 && c.cond_prec == 0 && !c.have_a32) {
    HIPCHK(&c, launch_cast_ahat(c));
    c.have_a32 = true;
  }
  if (inner_prec == HDG_BF16 && !c.have_a16) {
    HIPCHK(&c, launch_cast_ahat16(c));
    c.have_a16 = true;
  }
  *code = inner_prec == HDG_BF16 ? 2 : (inner_prec == HDG_FP32 ? 1 : 0);
  return HDG_OK;
}

hdg_status hdg_set_chunking(hdg_ctx ctx, int macros_per_chunk) {
  if (!ctx) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (macros_per_chunk < 0) return fail(&c, HDG_EINVAL, "macros_per_chunk must be >= 0");
  const int nm = c.hm.n_macros;
  const int per = (macros_per_chunk > 0 && macros_per_chunk < nm) ? macros_per_chunk : nm;
  if ((long long)((nm + per - 1) / per) * c.hm.n_classes + 1 > 4096)
    return fail(&c, HDG_EINVAL, "too many chunks (n_chunks * n_classes must stay below 4096)");
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  c.hm.chunk_macros = macros_per_chunk;
  plan_workspace(c);
  try {
    upload_w_offsets(c);
  } catch (const std::exception& ex) {
    return fail(&c, HDG_EDEVICE, ex.what());
  }
  // the previous binding no longer matches the layout
  c.ws_bound = false;
  c.lrn_bound = false;
  c.condensed64 = false;
  c.forget_w();
  c.store_valid = false;
  c.have_a32 = false;
  c.have_a16 = false;
  clear_graphs(c);
  return HDG_OK;
}

hdg_status hdg_set_chunk_buffers(hdg_ctx ctx, int n_buffers) {
  if (!ctx) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (n_buffers != 1 && n_buffers != 2) return fail(&c, HDG_EINVAL, "n_buffers must be 1 or 2");
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  c.hm.chunk_buffers = n_buffers;
  plan_workspace(c);
  try {
    upload_w_offsets(c);
  } catch (const std::exception& ex) {
    return fail(&c, HDG_EDEVICE, ex.what());
  }
  c.ws_bound = false;
  c.lrn_bound = false;
  c.condensed64 = false;
  c.forget_w();
  c.store_valid = false;
  c.have_a32 = false;
  c.have_a16 = false;
  clear_graphs(c);
  return HDG_OK;
}

hdg_status hdg_set_factor_store(hdg_ctx ctx, int n_macros, hdg_prec prec) {
  if (!ctx) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (n_macros < 0) return fail(&c, HDG_EINVAL, "n_macros must be >= 0");
  if (prec != HDG_FP64 && prec != HDG_FP32) return fail(&c, HDG_EUNSUPPORTED, "factor store precision not built");
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  c.hm.store_macros = n_macros;
  c.hm.store_prec = prec == HDG_FP32 ? 1 : 0;
  plan_workspace(c);
  try {
    upload_w_offsets(c);
  } catch (const std::exception& ex) {
    return fail(&c, HDG_EDEVICE, ex.what());
  }
  c.ws_bound = false;
  c.lrn_bound = false;
  c.condensed64 = false;
  c.forget_w();
  c.store_valid = false;
  c.have_a32 = false;
  c.have_a16 = false;
  clear_graphs(c);
  return HDG_OK;
}

hdg_status hdg_set_progress(hdg_ctx ctx, int on) {
  if (!ctx) return HDG_EINVAL;
  ctx->c.progress = on != 0;
  return HDG_OK;
}

hdg_status hdg_factor_store_macros(hdg_ctx ctx, int* n_stored) {
  if (!ctx || !n_stored) return HDG_EINVAL;
  const HostMesh& hm = ctx->c.hm;
  *n_stored = hm.store_chunks > 0 ? hm.chunk_first[hm.store_chunks] : 0;
  return HDG_OK;
}

hdg_status hdg_bind_workspace(hdg_ctx ctx, void* dev_ptr, size_t bytes) {
  if (!ctx || !dev_ptr) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (bytes < c.need_bytes) return fail(&c, HDG_ENOMEM, "workspace smaller than hdg_query_sizes().workspace_bytes");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) return fail(&c, HDG_EINVAL, "workspace must be 256-byte aligned");
  char* base = static_cast<char*>(dev_ptr);
  if (c.ws_bound) {
    // re-binding: offsets are relative to the previous base
    const char* old = c.ws.base;
    auto rebase = [&](auto*& p) { p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(base + (reinterpret_cast<const char*>(p) - old)); };
    rebase(c.ws.Kq); rebase(c.ws.AUU); rebase(c.ws.AUQ); rebase(c.ws.RUe); rebase(c.ws.RQe); rebase(c.ws.SUB);
    rebase(c.ws.RU); rebase(c.ws.RQ); rebase(c.ws.RQt); rebase(c.ws.RBloc); rebase(c.ws.RBglob); rebase(c.ws.gloc); rebase(c.ws.Wm);
    rebase(c.ws.ipiv); rebase(c.ws.FW); rebase(c.ws.fpiv); rebase(c.ws.A32); rebase(c.ws.A16); rebase(c.ws.ypart); rebase(c.ws.kry);
    rebase(c.ws.red); rebase(c.ws.small); rebase(c.ws.Uinv); rebase(c.ws.lrn); rebase(c.ws.kctl); rebase(c.ws.supg);
    rebase(c.ws.Ac); rebase(c.ws.bloc); rebase(c.ws.Fst);
  } else {
    auto rebase = [&](auto*& p) { p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(base + reinterpret_cast<uintptr_t>(p)); };
    rebase(c.ws.Kq); rebase(c.ws.AUU); rebase(c.ws.AUQ); rebase(c.ws.RUe); rebase(c.ws.RQe); rebase(c.ws.SUB);
    rebase(c.ws.RU); rebase(c.ws.RQ); rebase(c.ws.RQt); rebase(c.ws.RBloc); rebase(c.ws.RBglob); rebase(c.ws.gloc); rebase(c.ws.Wm);
    rebase(c.ws.ipiv); rebase(c.ws.FW); rebase(c.ws.fpiv); rebase(c.ws.A32); rebase(c.ws.A16); rebase(c.ws.ypart); rebase(c.ws.kry);
    rebase(c.ws.red); rebase(c.ws.small); rebase(c.ws.Uinv); rebase(c.ws.lrn); rebase(c.ws.kctl); rebase(c.ws.supg);
    rebase(c.ws.Ac); rebase(c.ws.bloc); rebase(c.ws.Fst);
  }
  c.ws.base = base;
  c.lrn_bound = false;
  clear_graphs(c);
  c.ws.bytes = bytes;
  c.ws_bound = true;
  c.have_a32 = false;
  c.have_a16 = false;
  c.linearized = false;
  c.condensed64 = false;
  c.forget_w();
  c.store_valid = false;
  return HDG_OK;
}

hdg_status hdg_autotune(hdg_ctx ctx, hdg_prec prec, const char* cache_path, int* n_timed) {
  if (!ctx) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  if (!c.linearized) return fail(&c, HDG_EINVAL, "autotune needs a linearisation (hdg_linearize_stage) first");
  if (prec != HDG_FP64 && prec != HDG_FP32) return fail(&c, HDG_EUNSUPPORTED, "condensation precision not built");
  const int p32 = prec == HDG_FP32 ? 1 : 0;
  c.condensed64 = false;  // the trials overwrite W (also when one fails)
  c.forget_w();
  c.store_valid = false;
  int dev = 0, rt = 0;
  HIPCHK(&c, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(&c, hipGetDeviceProperties(&prop, dev));
  HIPCHK(&c, hipRuntimeGetVersion(&rt));
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  // cache: one line per (arch, runtime, precision, class shape, batch):
  //   arch runtime prec dim m0 m1 m2 p batch | tpw panel lookahead ms
  std::map<std::string, LuTune> cache;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string a, pr;
      int r, d, m0, m1, m2, p, batch, tpw, wide, look;
      double ms;
      if (ls >> a >> r >> pr >> d >> m0 >> m1 >> m2 >> p >> batch >> tpw >> wide >> look >> ms) {
        std::ostringstream key;
        key << a << ' ' << r << ' ' << pr << ' ' << d << ' ' << m0 << ' ' << m1 << ' ' << m2 << ' ' << p << ' ' << batch;
        LuTune t;
        t.tpw = tpw;
        t.panel = wide;
        t.lookahead = look;
        if (tpw >= 4 && tpw <= 256 && tpw % 4 == 0 && wide >= 0 && wide <= 2 && (look == 0 || look == 1))
          cache[key.str()] = t;
      }
    }
  }
  const int ncl = c.hm.n_classes, nch = c.hm.n_chunks();
  int* status = reinterpret_cast<int*>(c.ws.small);
  hipEvent_t ev0, ev1;
  HIPCHK(&c, hipEventCreate(&ev0));
  HIPCHK(&c, hipEventCreate(&ev1));
  std::vector<std::string> fresh;
  int timed = 0;
  hdg_status st = HDG_OK;
  for (int k = 0; k < ncl && st == HDG_OK; ++k) {
    HostClass& h = c.hcs[k];
    int jbest = 0;  // the chunk holding most macros of the class
    for (int j = 1; j < nch; ++j)
      if (c.hm.chunk_class_cnt[(size_t)j * ncl + k] > c.hm.chunk_class_cnt[(size_t)jbest * ncl + k]) jbest = j;
    const int batch = c.hm.chunk_class_cnt[(size_t)jbest * ncl + k];
    std::ostringstream key;
    key << arch << ' ' << rt << ' ' << (p32 ? "fp32" : "fp64") << ' ' << h.dim << ' ' << h.m[0] << ' ' << h.m[1] << ' '
        << h.m[2] << ' ' << h.p << ' ' << batch;
    auto it = cache.find(key.str());
    if (it != cache.end()) {
      h.tune[p32] = it->second;
      continue;
    }
    // tiles per workgroup 8..256 with the default panel, then the wide panel
    // and the tournament with the best of those; one untimed trial first
    // (code loading)
    float best = 1e30f;
    LuTune pick;
    // then the look-ahead stream with the best so far
    constexpr int NCAND = 10;
    const int cand[NCAND][3] = {{32, 0, 0}, {8, 0, 0},  {16, 0, 0}, {32, 0, 0}, {64, 0, 0}, {128, 0, 0}, {256, 0, 0},
                                {-1, 1, 0}, {-1, 2, 0}, {-1, -1, 1}};
    for (int ci = 0; ci < NCAND && st == HDG_OK; ++ci) {
      {
        LuTune t;
        t.tpw = cand[ci][0] > 0 ? cand[ci][0] : pick.tpw;
        t.panel = cand[ci][1] >= 0 ? cand[ci][1] : pick.panel;
        t.lookahead = cand[ci][2];
        h.tune[p32] = t;
        float tmin = 1e30f;
        for (int rep = 0; rep < 1 && st == HDG_OK; ++rep) {
          hipError_t e = launch_zero_ints(c.stream, status, nch * ncl + 1);
          if (e == hipSuccess) e = launch_form(c, p32, c.hm.chunk_first[jbest], c.hm.chunk_first[jbest + 1], k);
          if (e == hipSuccess) e = hipEventRecord(ev0, c.stream);
          if (e == hipSuccess) e = launch_lu(c, p32, jbest, false, k);
          if (e == hipSuccess) e = hipEventRecord(ev1, c.stream);
          if (e == hipSuccess) e = hipEventSynchronize(ev1);
          float ms = 0.0f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
          if (e != hipSuccess) {
            st = fail(&c, HDG_EDEVICE, hipGetErrorString(e));
            break;
          }
          tmin = std::min(tmin, ms);
        }
        // another panel and the second stream only for a gain beyond the
        // spread of single timings (about 2%)
        const float need = (cand[ci][1] != 0 || cand[ci][2] != 0) ? 0.98f : 1.0f;
        if (ci > 0 && tmin < need * best) { best = tmin; pick = t; }
      }
    }
    h.tune[p32] = pick;
    ++timed;
    std::ostringstream line;
    line << key.str() << ' ' << pick.tpw << ' ' << pick.panel << ' ' << pick.lookahead << ' ' << best;
    fresh.push_back(line.str());
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (st != HDG_OK) return st;
  if (cache_path && !fresh.empty()) {
    std::ofstream out(cache_path, std::ios::app);
    for (const std::string& l : fresh) out << l << '\n';
    if (!out) return fail(&c, HDG_EINVAL, std::string("cannot write the tuning cache ") + cache_path);
  }
  if (n_timed) *n_timed = timed;
  // the trials overwrote the condensed matrices
  c.have_a32 = false;
  c.have_a16 = false;
  c.condensed64 = false;
  c.forget_w();
  c.store_valid = false;
  return HDG_OK;
}

hdg_status hdg_class_count(hdg_ctx ctx, int* n_classes) {
  if (!ctx || !n_classes) return HDG_EINVAL;
  *n_classes = ctx->c.hm.n_classes;
  return HDG_OK;
}

hdg_status hdg_set_tuning(hdg_ctx ctx, int macro_class, hdg_prec prec, int tpw, int panel, int lookahead) {
  if (!ctx || macro_class < 0 || macro_class >= ctx->c.hm.n_classes || (prec != HDG_FP64 && prec != HDG_FP32) ||
      tpw < 4 || tpw > 256 || tpw % 4 || panel < 0 || panel > 2 || (lookahead != 0 && lookahead != 1))
    return HDG_EINVAL;
  LuTune& t = ctx->c.hcs[macro_class].tune[prec == HDG_FP32 ? 1 : 0];
  t.tpw = tpw;
  t.panel = panel;
  t.lookahead = lookahead;
  return HDG_OK;
}

hdg_status hdg_get_tuning(hdg_ctx ctx, int macro_class, hdg_prec prec, int* tpw, int* panel, int* lookahead) {
  if (!ctx || macro_class < 0 || macro_class >= ctx->c.hm.n_classes || (prec != HDG_FP64 && prec != HDG_FP32))
    return HDG_EINVAL;
  const LuTune& t = ctx->c.hcs[macro_class].tune[prec == HDG_FP32 ? 1 : 0];
  if (tpw) *tpw = t.tpw;
  if (panel) *panel = t.panel;
  if (lookahead) *lookahead = t.lookahead;
  return HDG_OK;
}

hdg_status hdg_linearize_stage(hdg_ctx ctx, const double* q, const double* u, const double* uhat, const double* w,
                               double dt, double d_ii, double dtau, double norms_host[3]) {
  if (!ctx || !q || !u || !uhat) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  if (!(dt > 0) || !(dtau > 0) || std::isnan(d_ii)) return fail(&c, HDG_EINVAL, "dt and dtau must be positive");
  StageArgs sa{dt, d_ii, dtau};
  // the element blocks (and, chunked, W) change from here on
  c.condensed64 = false;
  c.forget_w();
  c.store_valid = false;
  c.have_a32 = false;
  c.have_a16 = false;
  HIPCHK(&c, launch_linearize(c, q, u, uhat, w, sa));
  c.linearized = true;
  if (norms_host) {
    HIPCHK(&c, launch_norms(c, c.ws.small + 2048));
    HIPCHK(&c, hipMemcpyAsync(ctx->pinned, c.ws.small + 2048, 3 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(&c, hipStreamSynchronize(c.stream));
    for (int i = 0; i < 3; ++i) norms_host[i] = ctx->pinned[i];
    if (!std::isfinite(norms_host[0] + norms_host[1] + norms_host[2])) return fail(&c, HDG_ENAN, "non-finite residual");
  }
  return HDG_OK;
}

// Formation, elimination and (chunked) extraction of every chunk.  With two
// slots, chunk j + 1 is formed on the formation stream into the other slot
// while chunk j is eliminated and extracted on the library's stream; a slot is
// formed again once the extraction of the chunk before has read it.
static hipError_t condense_chunks(HdgContext& c, int p32) {
  const int nch = c.hm.n_chunks();
  hipError_t e;
  if (c.hm.slots() < 2) {
    for (int j = 0; j < nch; ++j) {
      if ((e = launch_form(c, p32, c.hm.chunk_first[j], c.hm.chunk_first[j + 1])) != hipSuccess) return e;
      if ((e = launch_lu(c, p32, j, false)) != hipSuccess) return e;
      if ((e = launch_store_factors(c, p32, j)) != hipSuccess) return e;
      if (c.hm.chunked() && (e = launch_extract(c, p32, j)) != hipSuccess) return e;
      if ((e = report_progress(c, "condensation: chunk", j + 1, nch)) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if ((e = form_stream_ready(c)) != hipSuccess) return e;
  hipStream_t fs = c.form_stream;
  hipEvent_t* ev = c.form_events;  // [0] start, [1 + b] slot b formed, [3 + b] slot b free
  // the linearisation (whose element products share W) and earlier work come first
  if ((e = hipEventRecord(ev[0], c.stream)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(fs, ev[0], 0)) != hipSuccess) return e;
  auto form = [&](int j) -> hipError_t {
    hipError_t r;
    const int b = j % 2;
    if (j >= 2 && (r = hipStreamWaitEvent(fs, ev[3 + b], 0)) != hipSuccess) return r;
    if ((r = launch_form(c, p32, c.hm.chunk_first[j], c.hm.chunk_first[j + 1], -1, nullptr, fs)) != hipSuccess)
      return r;
    return hipEventRecord(ev[1 + b], fs);
  };
  if ((e = form(0)) != hipSuccess) return e;
  for (int j = 0; j < nch; ++j) {
    const int b = j % 2;
    if (j + 1 < nch && (e = form(j + 1)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(c.stream, ev[1 + b], 0)) != hipSuccess) return e;
    if ((e = launch_lu(c, p32, j, false)) != hipSuccess) return e;
    if ((e = launch_store_factors(c, p32, j)) != hipSuccess) return e;
    if ((e = launch_extract(c, p32, j)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev[3 + b], c.stream)) != hipSuccess) return e;
    if ((e = report_progress(c, "condensation: chunk", j + 1, nch)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hdg_status hdg_condense(hdg_ctx ctx, hdg_prec prec, double* bhat) {
  if (!ctx || !bhat) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  if (prec != HDG_FP64 && prec != HDG_FP32 && prec != HDG_BF16)
    return fail(&c, HDG_EINVAL, "unknown condensation precision");
  // HDG_BF16: FP32 storage, formation and panels; the trailing updates take
  // BF16 operands with FP32 accumulation
  const int p32 = (prec == HDG_FP32 || prec == HDG_BF16) ? 1 : 0;
  c.bf16_update = (prec == HDG_BF16);
  c.condensed64 = false;
  c.forget_w();
  c.store_valid = false;
  // status flags: one per (chunk, macro class), then one for the face blocks
  const int ncl = c.hm.n_classes, nch = c.hm.n_chunks(), nst = nch * ncl;
  int* status = reinterpret_cast<int*>(c.ws.small);
  HIPCHK(&c, launch_zero_ints(c.stream, status, nst + 1));
  HIPCHK(&c, condense_chunks(c, p32));
  HIPCHK(&c, launch_bhat(c, bhat, p32));
  HIPCHK(&c, launch_face_precond(c));
  c.cond_prec = p32;
  c.have_a32 = false;
  c.have_a16 = false;
  std::vector<int> st(nst + 1, 0);
  HIPCHK(&c, hipMemcpyAsync(ctx->pinned, status, sizeof(int) * (nst + 1), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  std::memcpy(st.data(), ctx->pinned, sizeof(int) * (nst + 1));
  for (int j = 0; j < nch; ++j)
    for (int k = 0; k < ncl; ++k) {
      const int v = st[(size_t)j * ncl + k];
      if (!v) continue;
      // the v-th macro of class k within chunk j (macros of a class in increasing order)
      int rank = v - 1, macro = -1;
      for (int i = c.hm.chunk_first[j]; i < c.hm.chunk_first[j + 1] && macro < 0; ++i)
        if (c.hm.macro_class[i] == k && rank-- == 0) macro = i;
      return fail(&c, HDG_ESINGULAR, "singular Schur complement in macro " + std::to_string(macro));
    }
  if (st[nst]) return fail(&c, HDG_ESINGULAR, "singular face block of A_uhat-uhat " + std::to_string(st[nst] - 1));
  c.condensed64 = (p32 == 0);
  if (c.hm.chunked())  // the last chunk of each slot
    for (int i = 0; i < c.hm.slots(); ++i) c.w_res[i] = nch - 1 - i;
  c.store_valid = c.hm.store_chunks > 0;
  return HDG_OK;
}

static hdg_status nested_get(hdg_ctx ctx, int block_m) {
  HdgContext& c = ctx->c;
  if (block_m < 1) return fail(&c, HDG_EINVAL, "block size must be positive");
  if (c.nested && c.nested_m == block_m) return HDG_OK;
  c.nested.reset();
  c.nested_m = 0;
  std::shared_ptr<NestedPlan> P;
  const std::string err = nested_plan(c, block_m, P);
  if (err.empty()) {
    c.nested = P;
    c.nested_m = block_m;
    return HDG_OK;
  }
  if (err.find("memory") != std::string::npos) return fail(&c, HDG_ENOMEM, err);
  if (err.find("multiple") != std::string::npos) return fail(&c, HDG_EINVAL, err);
  if (err.find("upload") != std::string::npos) return fail(&c, HDG_EDEVICE, err);
  return fail(&c, HDG_EUNSUPPORTED, err);
}

hdg_status hdg_nested_dims(hdg_ctx ctx, int block_m, int* n_blocks, int* n_internal, int* n_boundary) {
  if (!ctx) return HDG_EINVAL;
  const hdg_status s = nested_get(ctx, block_m);
  if (s != HDG_OK) return s;
  nested_dims(*ctx->c.nested, n_blocks, n_internal, n_boundary);
  return HDG_OK;
}

hdg_status hdg_condense_nested(hdg_ctx ctx, int block_m, double* ahat, double* bhat) {
  if (!ctx || !ahat || !bhat) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  if (!c.condensed64) return fail(&c, HDG_EINVAL, "nested condensation needs an FP64 hdg_condense of the current linearisation");
  const hdg_status s = nested_get(ctx, block_m);
  if (s != HDG_OK) return s;
  int singular = 0;
  HIPCHK(&c, launch_condense_nested(c, *c.nested, ahat, bhat, &singular));
  if (singular) return fail(&c, HDG_ESINGULAR, "singular internal-face block of nested block " + std::to_string(singular - 1));
  return HDG_OK;
}

static hdg_status fgmres_run(hdg_ctx ctx, Krylov& K, const double* b, double* x, const hdg_krylov_opts* o,
                             hdg_krylov_stats* st, std::chrono::steady_clock::time_point t0);

hdg_status hdg_nested_solve(hdg_ctx ctx, int block_m, double* x_full, const hdg_krylov_opts* o,
                            hdg_krylov_stats* st) {
  if (!ctx || !x_full || !o) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  if (!c.nested || c.nested_m != block_m || !nested_condensed(*c.nested))
    return fail(&c, HDG_EINVAL, "hdg_nested_solve needs hdg_condense_nested with the same block size first");
  if (o->restart < 1 || o->restart > c.kry_restart_max || o->inner_its < 0 || o->inner_its > c.kry_inner_max ||
      o->max_outer < 1 || !(o->rtol >= 0) || !(o->atol >= 0))
    return fail(&c, HDG_EINVAL, "bad Krylov options");
  if (o->use_learned || o->harvest_max || o->graph_steps || o->inner_prec != HDG_FP64)
    return fail(&c, HDG_EUNSUPPORTED, "the skeleton solve takes FP64 host-controlled steps only");
  const auto t0 = std::chrono::steady_clock::now();
  NestedPlan& P = *c.nested;
  const long long n = nested_skeleton_size(P);
  Krylov K(c, o->restart, o->inner_its, ctx->pinned, 0, n);
  K.opA = [&](const double* x, double* y) { return launch_nested_apply(c, P, x, y); };
  K.opM = [&](const double* v, double* z) { return launch_nested_jacobi(c, P, v, z); };
  const double* b = nested_rhs(P);
  double* x = nested_xskel(P);
  HIPCHK(&c, launch_scale_copy(c.stream, n, 0.0, b, x));  // zero start
  const hdg_status s = fgmres_run(ctx, K, b, x, o, st, t0);
  if (s != HDG_OK && s != HDG_ENOCONV) return s;
  // the internal traces (of the last iterate when max_outer was reached)
  HIPCHK(&c, launch_nested_recover(c, P, x, x_full));
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  if (st) st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return s;
}

hdg_status hdg_condense_first_layer(hdg_ctx ctx, double* bhat) {
  if (!ctx || !bhat) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  if (!c.hm.chunked() || c.hm.n_classes != 1)
    return fail(&c, HDG_EUNSUPPORTED, "first-layer condensation needs chunking and a single macro shape");
  c.forget_w();  // W holds the first-layer matrices from here on
  c.store_valid = false;
  int* status = reinterpret_cast<int*>(c.ws.small);
  const int nst = c.hm.n_chunks() * c.hm.n_classes;
  HIPCHK(&c, launch_zero_ints(c.stream, status, nst + 1));
  const hipError_t e = launch_condense_first_layer(c, status);
  if (e == hipErrorInvalidValue) return fail(&c, HDG_ENOMEM, "the W buffer cannot hold one first-layer matrix");
  if (e == hipErrorNotSupported)
    return fail(&c, HDG_EUNSUPPORTED, "first-layer matrix larger than the form and panel kernels take");
  HIPCHK(&c, e);
  HIPCHK(&c, launch_bhat(c, bhat, 0));
  HIPCHK(&c, launch_face_precond(c));
  c.cond_prec = 0;
  c.condensed64 = false;
  c.have_a32 = false;
  c.have_a16 = false;
  HIPCHK(&c, hipMemcpyAsync(ctx->pinned, status, sizeof(int) * (nst + 1), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  int st[2];
  std::memcpy(st, ctx->pinned, sizeof(int));
  std::memcpy(st + 1, reinterpret_cast<const int*>(ctx->pinned) + nst, sizeof(int));
  if (st[0]) return fail(&c, HDG_ESINGULAR, "singular first-layer local matrix");
  if (st[1]) return fail(&c, HDG_ESINGULAR, "singular face block of A_uhat-uhat " + std::to_string(st[1] - 1));
  return HDG_OK;
}

hdg_status hdg_flow_diagnostics(hdg_ctx ctx, const double* q, const double* u, double out_host[3]) {
  if (!ctx || !q || !u || !out_host) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  double* dev_out = c.ws.small + 2056;
  HIPCHK(&c, launch_flow_diagnostics(c, q, u, dev_out));
  HIPCHK(&c, hipMemcpyAsync(ctx->pinned, dev_out, 3 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  for (int i = 0; i < 3; ++i) out_host[i] = ctx->pinned[i];
  return HDG_OK;
}

hdg_status hdg_flow_diagnostics_noalloc(hdg_ctx ctx, const double* q, const double* u, double out_host[3]) {
  if (!ctx || !q || !u || !out_host) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  double* dev_out = nullptr;
  std::string err;
  hipError_t e = launch_flow_diagnostics_static(c, q, u, &dev_out, err);
  if (e != hipSuccess) return err.empty() ? hip_fail(&c, e, "flow diagnostics") : fail(&c, HDG_EINVAL, err);
  HIPCHK(&c, hipMemcpyAsync(ctx->pinned, dev_out, 3 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  for (int i = 0; i < 3; ++i) out_host[i] = ctx->pinned[i];
  return HDG_OK;
}

hdg_status hdg_apply_global(hdg_ctx ctx, const double* x, double* y) {
  if (!ctx || !x || !y || x == y) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  HIPCHK(&c, launch_apply(c, x, y, 0));
  return HDG_OK;
}

// FGMRES (Sec. 4.2) on the operator of K from the start x: the body of
// hdg_fgmres_solve, shared with the nested skeleton solve (whose K carries
// another operator and preconditioner; it takes no learned stage, harvest
// or graphs).
static hdg_status fgmres_run(hdg_ctx ctx, Krylov& K, const double* b, double* x, const hdg_krylov_opts* o,
                             hdg_krylov_stats* st, std::chrono::steady_clock::time_point t0) {
  HdgContext& c = ctx->c;
  // the learned stage is judged against the plain preconditioner of this
  // solve: the first LRN_JUDGE_STEPS steps run plain and measure its mean
  // residual reduction, then the learned stage is switched on
  const bool use_learned = o->use_learned != 0;
  const int judge_steps = use_learned ? LRN_JUDGE_STEPS : 0;
  K.learned = use_learned && judge_steps == 0;
  const long long n = K.n;
  int harvested = 0, fallbacks = 0;
  double lrn_log = 0.0, plain_log = 0.0;
  int lrn_steps = 0, plain_n = 0;
  double bnorm, beta;
  HIPCHK(&c, K.norm(b, bnorm));
  const double tol = std::max(o->rtol * bnorm, o->atol);
  HIPCHK(&c, K.apply_A(x, K.t, 0));
  HIPCHK(&c, launch_sub(c.stream, n, b, K.t, K.r));
  HIPCHK(&c, K.norm(K.r, beta));
  int its = 0;
  const int m = o->restart;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  // residual reduction |g_{j+1}| / |g_j| of one step (at most 1 in FGMRES):
  // plain steps feed this solve's mean plain rate; learned steps are compared
  // with it (fallback rule of the options)
  auto account = [&](bool step_learned, double rate) {
    if (!(rate > 0.0)) return;
    if (!step_learned) {
      plain_log += std::log(rate);
      ++plain_n;
      if (use_learned && !fallbacks && plain_n >= judge_steps) K.learned = true;
      return;
    }
    lrn_log += std::log(rate);
    ++lrn_steps;
    if (o->no_fallback) return;
    const bool worse_than_plain = lrn_steps >= 3 && plain_n >= 1 && lrn_log / lrn_steps > plain_log / plain_n;
    if (rate >= LRN_STAGNATION || worse_than_plain) {
      K.learned = false;
      fallbacks = 1;
    }
  };
  // steps left before the learned stage may switch on (graph batches stop there)
  auto judging_left = [&]() { return (use_learned && !fallbacks && !K.learned) ? judge_steps - plain_n : 0; };
  const bool dev_mode = o->graph_steps > 0 && o->harvest_max == 0;
  if (dev_mode) K.dev_init();
  while (beta > tol && its < o->max_outer) {
    HIPCHK(&c, launch_scale_copy(c.stream, n, 1.0 / beta, K.r, K.V));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    if (dev_mode) {
      // Arnoldi steps on the device, graph_steps at a time; the host only
      // reads |g_{j+1}| after each batch for the convergence test
      double* hb = ctx->pinned;
      for (int i = 0; i <= m; ++i) hb[i] = g[i];
      HIPCHK(&c, hipMemcpyAsync(K.dg, hb, sizeof(double) * (m + 1), hipMemcpyHostToDevice, c.stream));
      double prev = beta;
      bool done = false;
      int batch = o->graph_steps;
      for (int j = 0; j < m && !done;) {
        int kk = std::min(std::min(batch, m - j), o->max_outer - its);
        if (judging_left() > 0) kk = std::min(kk, judging_left());
        const double res_in = prev;
        const bool step_learned = K.learned;
        HIPCHK(&c, K.steps_graph(j, kk, m));
        HIPCHK(&c, hipMemcpyAsync(hb, K.dres + j, sizeof(double) * kk, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(&c, hipStreamSynchronize(c.stream));
        for (int jj = 0; jj < kk; ++jj) {
          const double res = hb[jj];
          ++its;
          k = j + jj + 1;
          account(step_learned, prev > 0.0 ? res / prev : 0.0);
          prev = res;
          if (!std::isfinite(res)) return fail(&c, HDG_ENAN, "non-finite Krylov residual");
          if (res <= tol || res == 0.0 || its >= o->max_outer) { done = true; break; }
        }
        j += kk;
        // next batch: the steps that the observed mean reduction per step still
        // needs to reach tol (at least 1, at most graph_steps), so that few
        // steps past convergence are computed
        if (!done && prev > 0.0 && res_in > 0.0 && prev < res_in) {
          const double rate = std::pow(prev / res_in, 1.0 / kk);
          const double need = std::ceil(std::log(tol / prev) / std::log(rate));
          batch = (int)std::max(1.0, std::min((double)o->graph_steps, need));
        } else {
          batch = o->graph_steps;
        }
      }
      // the k x k triangle of H and g to the host
      HIPCHK(&c, hipMemcpyAsync(hb, K.dH, sizeof(double) * (size_t)k * m, hipMemcpyDeviceToHost, c.stream));
      HIPCHK(&c, hipMemcpyAsync(hb + (size_t)k * m, K.dg, sizeof(double) * k, hipMemcpyDeviceToHost, c.stream));
      HIPCHK(&c, hipStreamSynchronize(c.stream));
      for (int i = 0; i < k; ++i) {
        g[i] = hb[(size_t)k * m + i];
        for (int j = 0; j < k; ++j) H[(size_t)i * m + j] = hb[(size_t)i * m + j];
      }
    }
    for (int j = 0; j < m && !dev_mode; ++j) {
      if (harvested < o->harvest_max) {
        HIPCHK(&c, hipMemcpyAsync(o->harvest + (size_t)harvested * n, K.V + (size_t)j * n, sizeof(double) * n,
                                  hipMemcpyDeviceToDevice, c.stream));
        ++harvested;
      }
      const bool step_learned = K.learned;
      HIPCHK(&c, K.precond(K.V + (size_t)j * n, K.Z + (size_t)j * n));
      double* wv = K.V + (size_t)(j + 1) * n;
      HIPCHK(&c, K.apply_A(K.Z + (size_t)j * n, wv, 0));
      double h[128];
      HIPCHK(&c, K.cgs2(K.V, j, wv, h));
      double hn;
      HIPCHK(&c, K.norm(wv, hn));
      for (int i = 0; i < j; ++i) {
        double a = h[i], bb = h[i + 1];
        h[i] = cs[i] * a + sn[i] * bb;
        h[i + 1] = -sn[i] * a + cs[i] * bb;
      }
      double rr = std::hypot(h[j], hn);
      cs[j] = rr > 0 ? h[j] / rr : 1.0;
      sn[j] = rr > 0 ? hn / rr : 0.0;
      h[j] = rr;
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
      double g0 = g[j];
      g[j] = cs[j] * g0;
      g[j + 1] = -sn[j] * g0;
      ++its;
      account(step_learned, std::fabs(g0) > 0.0 ? std::fabs(g[j + 1]) / std::fabs(g0) : 0.0);
      k = j + 1;
      if (hn == 0.0 || std::fabs(g[j + 1]) <= tol || its >= o->max_outer) break;
      HIPCHK(&c, launch_scale_copy(c.stream, n, 1.0 / hn, wv, wv));
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int j = i + 1; j < k; ++j) s -= H[(size_t)i * m + j] * y[j];
      y[i] = H[(size_t)i * m + i] != 0.0 ? s / H[(size_t)i * m + i] : 0.0;
    }
    for (int i = 0; i < k; ++i) ctx->pinned[i] = y[i];
    HIPCHK(&c, hipMemcpyAsync(K.dev_coef + 256, ctx->pinned, sizeof(double) * k, hipMemcpyHostToDevice, c.stream));
    HIPCHK(&c, launch_lincomb(c.stream, n, k, K.Z, n, K.dev_coef + 256, x, 1));
    HIPCHK(&c, K.apply_A(x, K.t, 0));
    HIPCHK(&c, launch_sub(c.stream, n, b, K.t, K.r));
    HIPCHK(&c, K.norm(K.r, beta));
    if (!std::isfinite(beta)) return fail(&c, HDG_ENAN, "non-finite Krylov residual");
  }
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  if (st) {
    st->outer_its = its;
    st->inner_its_total = K.inner_total;
    st->res0 = bnorm;
    st->res_final = beta;
    st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st->fallbacks = fallbacks;
    st->harvested = harvested;
  }
  if (beta > tol) return fail(&c, HDG_ENOCONV, "FGMRES reached max_outer");
  return HDG_OK;
}

hdg_status hdg_fgmres_solve(hdg_ctx ctx, const double* b, double* x, const hdg_krylov_opts* o, hdg_krylov_stats* st) {
  if (!ctx || !b || !x || !o) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  if (o->restart < 1 || o->restart > c.kry_restart_max || o->inner_its < 0 || o->inner_its > c.kry_inner_max ||
      o->max_outer < 1 || !(o->rtol >= 0) || !(o->atol >= 0) || o->graph_steps < 0)
    return fail(&c, HDG_EINVAL, "bad Krylov options");
  const auto t0 = std::chrono::steady_clock::now();
  int icode = 0;
  if (hdg_status s = inner_operator(c, o->inner_prec, &icode); s != HDG_OK) return s;
  if (o->use_learned && !c.lrn_bound) return fail(&c, HDG_EINVAL, "use_learned without a bound network");
  if (o->harvest_max < 0 || (o->harvest_max > 0 && !o->harvest)) return fail(&c, HDG_EINVAL, "bad harvest buffer");
  Krylov K(c, o->restart, o->inner_its, ctx->pinned, icode);
  return fgmres_run(ctx, K, b, x, o, st, t0);
}

hdg_status hdg_precond_apply(hdg_ctx ctx, const double* v, double* z, int inner_its, hdg_prec inner_prec,
                             int use_learned) {
  if (!ctx || !v || !z || v == z) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  if (inner_its < 0 || inner_its > c.kry_inner_max) return fail(&c, HDG_EINVAL, "bad inner_its");
  if (use_learned && !c.lrn_bound) return fail(&c, HDG_EINVAL, "use_learned without a bound network");
  int icode = 0;
  if (hdg_status s = inner_operator(c, inner_prec, &icode); s != HDG_OK) return s;
  Krylov K(c, 1, inner_its, ctx->pinned, icode);
  K.learned = use_learned != 0;
  HIPCHK(&c, K.precond(v, z));
  return HDG_OK;
}

hdg_status hdg_coarse_size(hdg_ctx ctx, int* n_features) {
  if (!ctx || !n_features) return HDG_EINVAL;
  *n_features = ctx->c.cd.cF;
  return HDG_OK;
}

hdg_status hdg_coarse_restrict(hdg_ctx ctx, const double* v, float* X) {
  if (!ctx || !v || !X) return HDG_EINVAL;
  HIPCHK(&ctx->c, launch_coarse_restrict(ctx->c, v, X));
  return HDG_OK;
}

hdg_status hdg_coarse_neighbours(hdg_ctx ctx, const float* X, float* Xe) {
  if (!ctx || !X || !Xe || X == Xe) return HDG_EINVAL;
  HIPCHK(&ctx->c, launch_coarse_neighbours(ctx->c, X, Xe));
  return HDG_OK;
}

hdg_status hdg_coarse_prolong(hdg_ctx ctx, const float* Y, double alpha, double* z) {
  if (!ctx || !Y || !z) return HDG_EINVAL;
  HIPCHK(&ctx->c, launch_coarse_prolong(ctx->c, Y, alpha, z));
  return HDG_OK;
}

size_t hdg_mlp_param_count(int n_in, int n_hidden, int n_out) {
  if (n_in <= 0 || n_hidden <= 0 || n_out <= 0) return 0;
  return mlp_param_count(n_in, n_hidden, n_out);
}

size_t hdg_mlp_work_floats(int n_in, int n_hidden, int n_out, int max_batch) {
  if (n_in <= 0 || n_hidden <= 0 || n_out <= 0 || max_batch <= 0) return 0;
  return mlp_work_floats(n_in, n_hidden, n_out, max_batch);
}

static bool mlp_ok(const hdg_mlp* net, int batch) {
  return net && net->params && net->work && net->n_in > 0 && net->n_hidden > 0 && net->n_out > 0 && batch > 0 &&
         batch <= net->max_batch;
}

hdg_status hdg_mlp_forward(hdg_ctx ctx, const hdg_mlp* net, const float* X, const int* idx, int batch, float* Y) {
  if (!ctx || !mlp_ok(net, batch) || !X || !Y) return HDG_EINVAL;
  HIPCHK(&ctx->c, launch_mlp_forward(ctx->c.stream, net->n_in, net->n_hidden, net->n_out, net->params, net->work, X,
                                     idx, batch, Y));
  return HDG_OK;
}

hdg_status hdg_mlp_loss_grad(hdg_ctx ctx, const hdg_mlp* net, const float* X, const float* T, const int* idx,
                             int batch, float* loss_dev) {
  if (!ctx || !mlp_ok(net, batch) || !net->grads || !X || !T) return HDG_EINVAL;
  HIPCHK(&ctx->c, launch_mlp_loss_grad(ctx->c.stream, net->n_in, net->n_hidden, net->n_out, net->params, net->grads,
                                       net->work, X, T, idx, batch, loss_dev));
  return HDG_OK;
}

hdg_status hdg_mlp_adam(hdg_ctx ctx, const hdg_mlp* net, float lr, float beta1, float beta2, float eps, int step) {
  if (!ctx || !net || !net->params || !net->grads || !net->adam_m || !net->adam_v || step < 1 || !(lr > 0) ||
      !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return HDG_EINVAL;
  const long long n = (long long)mlp_param_count(net->n_in, net->n_hidden, net->n_out);
  HIPCHK(&ctx->c, launch_mlp_adam(ctx->c.stream, n, net->params, net->grads, net->adam_m, net->adam_v, lr, beta1,
                                  beta2, eps, step));
  return HDG_OK;
}

hdg_status hdg_learned_bind(hdg_ctx ctx, const hdg_mlp* net) {
  if (!ctx) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!net) {
    c.lrn_bound = false;
    return HDG_OK;
  }
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  const int F = c.cd.cF, Fe = (1 + 2 * c.cd.dim) * F;
  if (!net->params || (net->n_in != F && net->n_in != Fe) || net->n_out != F || net->n_hidden <= 0 ||
      net->n_hidden > LRN_MAX_HIDDEN)
    return fail(&c, HDG_EINVAL, "network shape does not match the coarse space (or n_hidden > 512)");
  unsigned short* q = const_cast<unsigned short*>(learned_weights(c));
  HIPCHK(&c, launch_to_bf16(c.stream, (long long)mlp_param_count(net->n_in, net->n_hidden, net->n_out), net->params, q));
  // captured FGMRES steps hold the inference launch shape of the old network
  if (c.lrn_hidden != net->n_hidden || c.lrn_in != net->n_in) clear_graphs(c);
  c.lrn_hidden = net->n_hidden;
  c.lrn_in = net->n_in;
  c.lrn_bound = true;
  return HDG_OK;
}

hdg_status hdg_local_backsolve(hdg_ctx ctx, const double* duhat, double* dq, double* du) {
  if (!ctx || !duhat || !dq || !du) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return fail(&c, HDG_ENOMEM, "no workspace bound");
  HIPCHK(&c, launch_backsolve(c, duhat, dq, du));
  return HDG_OK;
}

hdg_status hdg_axpy(hdg_ctx ctx, size_t n, double a, const double* x, double* y) {
  if (!ctx || !x || !y) return HDG_EINVAL;
  HIPCHK(&ctx->c, launch_axpy(ctx->c.stream, n, a, x, y));
  return HDG_OK;
}

hdg_status hdg_destroy(hdg_ctx ctx) {
  if (!ctx) return HDG_EINVAL;
  (void)hipStreamSynchronize(ctx->c.stream);
  clear_graphs(ctx->c);
  if (ctx->c.cap_stream) (void)hipStreamDestroy(ctx->c.cap_stream);
  for (auto s : ctx->c.lu_streams) (void)hipStreamDestroy(s);
  for (auto ev : ctx->c.lu_events) (void)hipEventDestroy(ev);
  for (auto s : ctx->c.lu_pstreams) (void)hipStreamDestroy(s);
  for (auto ev : ctx->c.lu_pevents) (void)hipEventDestroy(ev);
  if (ctx->c.form_stream) (void)hipStreamDestroy(ctx->c.form_stream);
  for (auto ev : ctx->c.form_events)
    if (ev) (void)hipEventDestroy(ev);
  for (void* p : ctx->c.dev_allocs) (void)hipFree(p);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return HDG_OK;
}

// one tiled macro matrix to the host, widened to double if stored in FP32
static hdg_status copy_tiled_macro(hdg_ctx ctx, size_t macro, std::vector<double>& out, int prec) {
  HdgContext& c = ctx->c;
  const long long ws = c.hcs[c.hm.macro_class[macro]].wstride;
  const long long wo = c.hm.w_off[macro];
  out.assign((size_t)ws, 0.0);
  if (prec == 1) {
    std::vector<float> f((size_t)ws);
    HIPCHK(&c, hipMemcpyAsync(f.data(), reinterpret_cast<const float*>(c.ws.Wm) + wo, sizeof(float) * ws,
                              hipMemcpyDeviceToHost, c.stream));
    HIPCHK(&c, hipStreamSynchronize(c.stream));
    for (size_t i = 0; i < f.size(); ++i) out[i] = f[i];
    return HDG_OK;
  }
  HIPCHK(&c, hipMemcpyAsync(out.data(), c.ws.Wm + wo, sizeof(double) * ws, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(&c, hipStreamSynchronize(c.stream));
  return HDG_OK;
}

hdg_status hdg_get_condensed(hdg_ctx ctx, size_t macro, double* ahat_host, double* bhat_host) {
  if (!ctx) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound || macro >= (size_t)c.hm.n_macros) return HDG_EINVAL;
  const HostClass& hk = c.hcs[c.hm.macro_class[macro]];
  const int nb = hk.n_b, nu = hk.n_u;
  if (c.hm.chunked()) {  // compact copies
    const long long ao = c.hm.a32_off[macro], n2 = (long long)nb * nb;
    if (ahat_host && c.cond_prec == 1) {
      std::vector<float> f((size_t)n2);
      HIPCHK(&c, hipMemcpyAsync(f.data(), reinterpret_cast<const float*>(c.ws.Ac) + ao, sizeof(float) * n2,
                                hipMemcpyDeviceToHost, c.stream));
      HIPCHK(&c, hipStreamSynchronize(c.stream));
      for (long long i = 0; i < n2; ++i) ahat_host[i] = f[i];
    } else if (ahat_host) {
      HIPCHK(&c, hipMemcpyAsync(ahat_host, c.ws.Ac + ao, sizeof(double) * n2, hipMemcpyDeviceToHost, c.stream));
    }
    if (bhat_host)
      HIPCHK(&c, hipMemcpyAsync(bhat_host, c.ws.bloc + c.hm.b_off[macro], sizeof(double) * nb, hipMemcpyDeviceToHost,
                                c.stream));
    HIPCHK(&c, hipStreamSynchronize(c.stream));
    return HDG_OK;
  }
  std::vector<double> tiled;
  hdg_status s = copy_tiled_macro(ctx, macro, tiled, c.cond_prec);
  if (s != HDG_OK) return s;
  std::vector<double> g(nb, 0.0);  // FP32 condensation keeps g in FP64 outside W
  if (c.cond_prec == 1) {
    HIPCHK(&c, hipMemcpyAsync(g.data(), c.ws.gloc + c.hm.b_off[macro], sizeof(double) * nb, hipMemcpyDeviceToHost,
                              c.stream));
    HIPCHK(&c, hipStreamSynchronize(c.stream));
  }
  for (int r = 0; r < nb; ++r) {
    if (ahat_host)
      for (int k = 0; k < nb; ++k) ahat_host[(size_t)r * nb + k] = tiled[wtix(nu + r, nu + k, hk.ldw)];
    if (bhat_host) bhat_host[r] = g[r] + tiled[wtix(nu + r, hk.n_cols - 1, hk.ldw)];
  }
  return HDG_OK;
}

hdg_status hdg_get_formed(hdg_ctx ctx, size_t macro, double* w_host) {
  if (!ctx || !w_host) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound || macro >= (size_t)c.hm.n_macros) return HDG_EINVAL;
  int j = 0;  // the chunk holding the macro
  while (c.hm.chunk_first[j + 1] <= (int)macro) ++j;
  c.forget_w();  // W no longer holds a chunk's elimination
  HIPCHK(&c, launch_form(c, 0, c.hm.chunk_first[j], c.hm.chunk_first[j + 1]));
  if (!c.hm.chunked()) {  // W no longer holds the condensed operator
    c.cond_prec = 0;
    c.condensed64 = false;
  }
  std::vector<double> tiled;
  hdg_status s = copy_tiled_macro(ctx, macro, tiled, 0);
  if (s != HDG_OK) return s;
  const HostClass& hk = c.hcs[c.hm.macro_class[macro]];
  for (int r = 0; r < hk.n_rows; ++r)
    for (int k = 0; k < hk.n_cols; ++k) w_host[(size_t)r * hk.n_cols + k] = tiled[wtix(r, k, hk.ldw)];
  return HDG_OK;
}

hdg_status hdg_get_residuals(hdg_ctx ctx, double* rq, double* ru, double* rb) {
  if (!ctx) return HDG_EINVAL;
  HdgContext& c = ctx->c;
  if (!c.ws_bound) return HDG_EINVAL;
  if (rq) HIPCHK(&c, hipMemcpyAsync(rq, c.ws.RQ, sizeof(double) * c.n_q_tot, hipMemcpyDeviceToDevice, c.stream));
  if (ru) HIPCHK(&c, hipMemcpyAsync(ru, c.ws.RU, sizeof(double) * c.n_u_tot, hipMemcpyDeviceToDevice, c.stream));
  if (rb) HIPCHK(&c, hipMemcpyAsync(rb, c.ws.RBglob, sizeof(double) * c.md.n_glob, hipMemcpyDeviceToDevice, c.stream));
  return HDG_OK;
}

}  // extern "C"

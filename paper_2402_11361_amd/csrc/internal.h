// Internal declarations shared by the host runtime and the HIP kernels of
// libhdg.so.  Nothing here is part of the public ABI (include/hdg.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#define HDG_MAXD 3
#define HDG_MAXF 6

// Reference tables of one macro shape (m per axis, degree p, element sizes h),
// all device pointers.  A mesh may hold several shapes (classes); every
// macro refers to its class through MeshDev::macro_class.  Element-local node index a = a_0 + (p+1)(a_1 + (p+1)a_2);
// quadrature index q likewise with nq = p + 2 Gauss points per direction.
struct ClassDev {
  int dim, p, nq, ns;
  int m[3], n1[3];
  int N, E, A, Q, T, Fq;
  int n_u, n_q, n_b;
  int nf_nodes[HDG_MAXF];  // trace nodes per local macro face
  int nf_off[HDG_MAXF];    // dof offset of each local face in the macro trace vector
  int n_sub;               // sub-faces (element faces on the macro boundary)
  int nmax1;               // max n1
  double h[3];
  // element tables
  const double* Phi;   // [Q][A]
  const double* dPhi;  // [dim][Q][A] physical derivatives
  const double* W;     // [Q] weights times Jacobian
  const double* Tvol;  // [dim*Q][A*A]: -dPhi_k[q][a] * Phi[q][b]
  const double* Mel;   // [A][A] element mass matrix
  // face tables per local face lf (normal axis lf/2, side lf%2)
  const double* Psi;   // [2d][Fq][T] trace basis at face quadrature points
  const double* WF;    // [2d][Fq]
  const int* fnode;    // [2d][T] element-local node of face node t
  const int* finv;     // [2d][A] face node index t of element node a on local face lf, or -1
  // topology
  const int* elem_nodes;  // [E][A] macro node ids
  const int* elem_sub;    // [E][2d] sub-face id or -1
  const int* sub_elem;    // [n_sub]
  const int* sub_lf;      // [n_sub]
  const int* sub_tid;     // [n_sub][T] trace node ids on the macro face
  const int* node_ne;     // [N] number of elements containing the node
  const int* node_e;      // [N][8]
  const int* node_a;      // [N][8]
  const int* tn_cnt;      // [sum nf] sub-faces containing a trace node (per local face, concatenated)
  const int* tn_sub;      // [sum nf][4]
  const int* tn_t;        // [sum nf][4]
  const int* tn_base;     // [2d] offset of each local face in the tn_ arrays
  // 1D macro operators per axis (physical): C1D_k = M_k^{-1} B_k, Minv1D_k = M_k^{-1}
  const double* C1D;      // [dim][nmax1][nmax1]
  const double* Minv1D;   // [dim][nmax1][nmax1]
  const double* M1D;      // [dim][nmax1][nmax1]
  const double* B1D;      // [dim][nmax1][nmax1]: B_k[a][b] = int phi_b d_k phi_a (= M1D_k C1D_k)
  // coarse multilinear space on the macro faces (learned correction):
  // cq = 2^(d-1) functions per face and component, cF = 2d ns cq features per
  // macro, tables per normal axis k over the face nodes (lower axis fastest)
  int cq, cF, cmaxf;
  const double* cR;       // [dim][cq][cmaxf] discrete L2 projection (G^{-1} Phi^T W)
  const double* cPhi;     // [dim][cmaxf][cq] coarse functions at the face nodes
  // tiled augmented matrix of the class
  int ldw, n_rows, n_cols;
  long long wstride;      // elements per matrix
};

struct PhysDev {
  double gamma, Pr, Re, Mach, mu, Re_c, kappa;  // kappa = mu / (Re_c Pr (gamma-1))
  int supg;
};

// Per-Newton-step scalars of the linearisation.
struct StageArgs {
  double dt, dii, dtau;   // dt = inf: steady; dtau = inf: no continuation
};

// Device view of the mesh and workspace used by the kernels.
struct MeshDev {
  int dim, ns, n_macros, n_faces;
  long long n_glob;
  const int* macro_face;   // [n_macros][2d] global face id
  const int* macro_bnd;    // [n_macros][2d] 1 = Dirichlet face
  const long long* face_off;   // [n_faces] offset in the trace vector
  const int* face_ndof;        // [n_faces]
  const int* face_minus;       // [n_faces] macro on the low side or -1
  const int* face_plus;        // [n_faces] macro on the high side or -1
  const double* bc_state;      // [n_glob] Dirichlet data (or null)
  // macro classes and per-macro offsets (variable macro sizes)
  const ClassDev* cls;         // [n_classes]
  const int* macro_class;      // [n_macros]
  const long long* u_off;      // [n_macros + 1] offset of the macro in u (and R_U); q offsets are dim * u_off
  const long long* b_off;      // [n_macros + 1] offset in per-macro trace vectors (R_Uhat^(i), g, partial products)
  const long long* el_off;     // [n_macros + 1] first global element
  const int* elem_macro;       // [n_elements]
  const long long* sub_off;    // [n_macros + 1] first global sub-face
  const long long* row_off;    // [n_macros + 1] first row of the macro in the list of all augmented rows
  const long long* w_off;      // [n_macros] offset (elements) of the macro's tiled matrix, grouped by class
  const long long* ipiv_off;   // [n_macros] offset of the macro's pivot rows in the pivot array
  const long long* a32_off;    // [n_macros + 1] offset of the macro's compact FP32 copy of A-hat
  const int* face_slot;        // [n_faces] slot of the face's preconditioner block (grouped by size)
};

__device__ __forceinline__ const ClassDev& class_of(const MeshDev& md, int macro) {
  return md.cls[md.macro_class[macro]];
}

// largest i in [0, n) with off[i] <= g (off ascending, off[0] = 0)
__device__ __forceinline__ int find_in(const long long* off, int n, long long g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (off[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Storage of the augmented macro matrices (and of the face-preconditioner
// blocks): 16 x 64 tiles, each tile contiguous and row-major, tiles ordered
// row-major; ld is the padded width (a multiple of 64) and the row count is
// padded to a multiple of 16.  A 16-row slab of a 64-column strip is one
// contiguous 8 KB block, which keeps the MFMA trailing update streaming.
__host__ __device__ __forceinline__ size_t wtix(long long r, long long c, long long ld) {
  return ((size_t)(r >> 4) * (size_t)(ld >> 6) + (size_t)(c >> 6)) * 1024 + (size_t)(r & 15) * 64 + (size_t)(c & 63);
}

// Launch choices of the batched elimination, picked per macro class and
// precision by hdg_autotune: tpw = 16-row tiles per workgroup of the
// trailing update (4 waves); panel = how a block's pivots are found: 0 the
// one-workgroup register panel (512 threads), 1 the same with 1024 threads
// (fewer rows per thread), 2 tournament pivoting over groups of 256 rows;
// lookahead = the next pair's factorisation on a second stream beside the
// trailing update.
struct LuTune {
  int tpw = 32;
  int panel = 2;
  int lookahead = 0;
  int bf16_update = 0;  // FP32 storage: trailing update with BF16 operands, FP32 accumulation
};

// ---- kernel launchers (defined in the .hip files) ----------------------
struct Workspace;
struct HdgContext;

hipError_t launch_linearize(HdgContext& c, const double* q, const double* u, const double* uhat,
                            const double* w, StageArgs sa);
// prec: 0 FP64, 1 FP32 element type of the augmented matrices
// formation and elimination of the macros [m0, m1) = chunk j (rows of the
// trace block skipped in the elimination when top_only)
// rhs_duhat non-null: recovery form (S rows with f + C duhat in column n_u);
// on stream s (null: the library's stream)
hipError_t launch_form(HdgContext& c, int prec, int m0, int m1, int only_class = -1,
                       const double* rhs_duhat = nullptr, hipStream_t s = nullptr);
// chunks in two slots of W: the formation stream and its events
hipError_t form_stream_ready(HdgContext& c);
// with progress reporting on: waits for the library's stream and prints
// "<what> <i> of <n> done" on stderr
hipError_t report_progress(HdgContext& c, const char* what, int i, int n);
// top_only: eliminate the S rows only; rhs_only (with top_only): the columns
// [0, n_u] only (the recovery form's right-hand side in column n_u)
hipError_t launch_lu(HdgContext& c, int prec, int chunk, bool top_only, int only_class = -1, bool rhs_only = false);
// chunked condensation: A-hat^{T_i} and b-hat^{T_i} of chunk j out of W
hipError_t launch_extract(HdgContext& c, int prec, int chunk);
// chunked condensation: the factors of S of chunk j into the factor store
// (nothing for chunks it does not keep)
hipError_t launch_store_factors(HdgContext& c, int prec, int chunk);
hipError_t launch_bhat(HdgContext& c, double* bhat, int prec);
hipError_t launch_face_precond(HdgContext& c);
hipError_t launch_apply(HdgContext& c, const double* x, double* y, int prec);
hipError_t launch_precond_apply(HdgContext& c, const double* x, double* y);
hipError_t launch_backsolve(HdgContext& c, const double* duhat, double* dq, double* du);
hipError_t launch_axpy(hipStream_t s, size_t n, double a, const double* x, double* y);
hipError_t launch_norms(HdgContext& c, double* out3_dev);
hipError_t launch_supg(HdgContext& c, const double* q, const double* u, const double* w, StageArgs sa);
size_t supg_scratch_per_element(int dim, int p);
hipError_t launch_cast_ahat(HdgContext& c);
hipError_t launch_cast_ahat16(HdgContext& c);
// first-layer condensation (chunked workspace, one macro class)
hipError_t launch_condense_first_layer(HdgContext& c, int* status);
hipError_t launch_flow_diagnostics(HdgContext& c, const double* q, const double* u, double* out3_dev);
hipError_t diag_scratch_setup(int device);
hipError_t launch_flow_diagnostics_static(HdgContext& c, const double* q, const double* u, double** out3_dev,
                                          std::string& err);

// learned coarse correction
constexpr int LRN_MAX_HIDDEN = 512;
// learned-stage judge: plain FGMRES steps at the start of a solve that give
// the plain mean reduction, and the per-step reduction counted as stagnation
constexpr int LRN_JUDGE_STEPS = 3;
constexpr double LRN_STAGNATION = 0.99;
size_t mlp_param_count(int n_in, int n_hidden, int n_out);
size_t mlp_work_floats(int n_in, int n_hidden, int n_out, int max_batch);
hipError_t launch_coarse_restrict(HdgContext& c, const double* v, float* X);
hipError_t launch_coarse_prolong(HdgContext& c, const float* Y, double alpha, double* z);
hipError_t launch_coarse_neighbours(HdgContext& c, const float* X, float* Xe);
hipError_t launch_mlp_forward(hipStream_t s, int n_in, int n_hidden, int n_out, const float* params, float* work,
                              const float* X, const int* idx, int batch, float* Y);
hipError_t launch_mlp_loss_grad(hipStream_t s, int n_in, int n_hidden, int n_out, const float* params, float* grads,
                                float* work, const float* X, const float* T, const int* idx, int batch, float* loss);
hipError_t launch_mlp_adam(hipStream_t s, long long n, float* p, const float* g, float* m, float* v, float lr,
                           float b1, float b2, float eps, int t);
hipError_t launch_to_bf16(hipStream_t s, long long n, const float* p, unsigned short* q);
hipError_t launch_learned_correction(HdgContext& c, const double* v, double* z);
const unsigned short* learned_weights(const HdgContext& c);

// vector kernels for the Krylov solver
hipError_t launch_multidot(hipStream_t s, long long n, int k, const double* V, long long ldv,
                           const double* w, double* partial, double* out);
hipError_t launch_multiaxpy(hipStream_t s, long long n, int k, const double* V, long long ldv,
                            const double* coef, double sign, double* w);
hipError_t launch_scale_copy(hipStream_t s, long long n, double a, const double* x, double* y);
hipError_t launch_lincomb(hipStream_t s, long long n, int k, const double* V, long long ldv,
                          const double* coef_dev, double* y, int accumulate);
hipError_t launch_sub(hipStream_t s, long long n, const double* a, const double* b, double* y);
// device-resident Krylov control
hipError_t launch_accum_col(hipStream_t s, int n, const double* coef, double* col, int stride, int pass);
hipError_t launch_norm_finish(hipStream_t s, const double* dot, double* h_out, double* inv_out);
hipError_t launch_scale_dev(hipStream_t s, long long n, const double* a, const double* x, double* y);
hipError_t launch_givens_step(hipStream_t s, int j, int m, double* H, double* cs, double* sn, double* g, double* res);
hipError_t launch_small_ls(hipStream_t s, int k, int ldh, const double* Hin, const double* beta, double* y);

/*
 * hdg.h — C ABI of libhdg.so, the MI355X (gfx950) hot path of the matrix-free
 * macro-element HDG method for compressible Navier-Stokes
 * (Badrkhani, ten Eikelder, Hiemstra, Schillinger, arXiv 2402.11361).
 *
 * One Newton step of a DIRK stage (Sec. 3, Algorithm 1) is
 *     hdg_linearize_stage -> hdg_condense -> hdg_fgmres_solve
 *     (hdg_apply_global inside) -> hdg_local_backsolve -> hdg_axpy (update).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers owned by the caller (e.g. torch
 *     tensors) unless the name ends in _host.  They must stay valid until the
 *     work queued on the context's stream has finished.
 *   - Work is queued on the HIP stream given at setup, in call order.  Only
 *     calls with a _host output or a stats struct synchronise.
 *   - Errors are returned as hdg_status; the call then has no effect on its
 *     outputs unless stated, and hdg_last_error(ctx) gives a message.
 *     Invalid arguments give HDG_EINVAL before anything is queued.
 *   - Layouts (FP64 at the boundary always):
 *       u     [macro][comp][node]         comp = rho, rho v_1..v_d, rho E
 *       q     [macro][dir][comp][node]    q = grad u (eq. C4)
 *       uhat  [face][comp][facenode]      trace on the macro skeleton
 *     Macros may differ in size (segment lengths per axis): macro i starts at
 *     u_off[i] in u and at dim * u_off[i] in q (hdg_macro_offsets).
 *     Macros are numbered s_0 + n_seg0 (s_1 + n_seg1 s_2); macro nodes
 *     i_0 + n_0 (i_1 + n_1 i_2) with n_k = m_k p + 1 (GLL points in every
 *     element, C0 inside the macro).  Faces: all faces normal to axis 0, then
 *     1, then 2; within an axis lexicographic over the face grid (positions
 *     along the normal axis, macro segments along the others), axis 0
 *     fastest; face nodes over the tangential axes in increasing order.
 *   - Calls on one context are not thread safe.
 */
#ifndef HDG_H
#define HDG_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hdg_ctx_s* hdg_ctx;

typedef enum {
  HDG_OK = 0,
  HDG_EINVAL = 1,       /* bad argument (null, size, layout)                  */
  HDG_ENOMEM = 2,       /* workspace missing or too small                     */
  HDG_EDEVICE = 3,      /* HIP runtime error (message has the HIP string)     */
  HDG_ESINGULAR = 4,    /* zero pivot in a local factorisation                */
  HDG_ENOCONV = 5,      /* Krylov solve hit its iteration limit               */
  HDG_EBREAKDOWN = 6,   /* Krylov breakdown                                   */
  HDG_ENAN = 7,         /* non-finite residual                                */
  HDG_EUNSUPPORTED = 8  /* configuration not built (dimension, degree, ...)  */
} hdg_status;

typedef enum { HDG_FP64 = 0, HDG_FP32 = 1, HDG_BF16 = 2 } hdg_prec;

/* Box mesh on [lo, hi] with n_elem[k] uniform elements per axis, grouped into
 * box macro-elements: along axis k the segments have seg_len[k][0..n_seg[k])
 * elements (host arrays, summing to n_elem[k]; lengths may differ, giving
 * macros of several shapes, each shape one class of reference tables).
 * Degree p in every element (p = 1..3).
 * dim = 2 or 3.  Paper Sec. 2.2 (mesh, patches, spaces). */
typedef struct {
  int dim;
  int n_elem[3];
  double lo[3], hi[3];
  int periodic[3];
  int n_seg[3];
  const int* seg_len[3];
  int p;
} hdg_mesh_desc;

/* Physics (Sec. 2.1, acoustic scaling): Re_c = Re / Mach, mu = 1.
 * supg: 1 adds the SUPG term of eq. (C38b).  bc_state_host: global trace
 * vector (n_glob values, host) holding the Dirichlet state on boundary faces
 * (read at setup; may be NULL when every axis is periodic). */
typedef struct {
  double gamma, Pr, Re, Mach;
  int supg;
  const double* bc_state_host;
} hdg_phys;

typedef struct {
  size_t n_macros;     /* number of macro-elements                           */
  size_t n_glob;       /* global trace unknowns (length of uhat)             */
  size_t n_u_tot;      /* length of u                                        */
  size_t n_q_tot;      /* length of q                                        */
  size_t n_u_macro;    /* u unknowns per macro (n_s N), largest macro        */
  size_t n_b_macro;    /* trace unknowns on a macro's boundary, largest macro */
  size_t workspace_bytes; /* device workspace needed by hdg_bind_workspace   */
  size_t n_faces;      /* macro faces (entries of face_off)                  */
} hdg_sizes;

/* Krylov options (Sec. 4.2): outer right-preconditioned FGMRES(restart) whose
 * preconditioner is inner_its steps of GMRES left-preconditioned by the
 * inverse face blocks of A_uhat-uhat.  Convergence: ||b - A x||_2 <=
 * max(rtol ||b||_2, atol).  inner_prec selects the precision of the condensed
 * blocks used inside the preconditioner: HDG_FP32 after an FP64 condensation
 * uses an FP32 copy of A-hat there (made on first use); after an FP32
 * condensation both levels use the FP32 blocks.  HDG_BF16: a BF16 copy of
 * A-hat (rounded to nearest even, made on first use, applied with FP64
 * sums) inside the preconditioner only; the outer FGMRES keeps the
 * condensed operator, so the solution is unaffected (FGMRES admits a
 * preconditioner that differs from the operator), only iteration counts
 * change.  With chunked condensation: HDG_FP32 needs an FP32 condensation
 * and HDG_BF16 is HDG_EUNSUPPORTED. */
typedef struct {
  double rtol, atol;
  int restart, max_outer, inner_its;
  hdg_prec inner_prec;
  /* 1: add the learned coarse correction bound by hdg_learned_bind to the
   * preconditioner.  The plain preconditioner is the judge: the first 3
   * steps of the solve run plain and give the mean per-step residual
   * reduction |g_{j+1}| / |g_j| of this operator; then the learned stage is
   * switched on, and it falls back to the plain preconditioner for the rest
   * of the solve once its mean reduction over at least 3 steps is worse than
   * the plain mean, or once one of its steps reduces the residual by less
   * than 1% (ratio >= 0.99). */
  int use_learned;
  /* 1: keep the learned stage for the whole solve (no fallback; for
   * measuring what the network gains or loses on its own). */
  int no_fallback;
  /* optional (device, may be NULL): the vectors the preconditioner is
   * applied to are copied here, harvest_max vectors of n_glob doubles at
   * most, in the order they occur (training data of the learned stage). */
  double* harvest;
  int harvest_max;
  /* 0: Arnoldi control on the host (one synchronisation per Gram-Schmidt
   * pass).  k >= 1: the whole Arnoldi step (inner GMRES with its small
   * least-squares solve, CGS2, normalisation, Givens update) stays on the
   * device; each step is captured once per context in a HIP graph and
   * replayed; up to k steps are launched between two synchronisations (the
   * convergence test), fewer when the observed reduction per step says
   * fewer will reach the tolerance; steps past convergence in a batch are
   * computed and discarded.  Not combined with harvest (k is ignored while
   * harvesting). */
  int graph_steps;
} hdg_krylov_opts;

typedef struct {
  int outer_its, inner_its_total;
  double res0, res_final;
  double ms;
  int fallbacks;   /* 1 if the learned stage was switched off during the solve */
  int harvested;   /* vectors written to opts.harvest */
} hdg_krylov_stats;

/* Build the mesh topology, the reference tables of every macro shape and the
 * face tables; queue uploads on `hip_stream` (a hipStream_t, NULL = default).
 * Returns HDG_EINVAL for an inconsistent description. */
hdg_status hdg_setup_mesh(const hdg_mesh_desc* mesh, const hdg_phys* phys, void* hip_stream,
                          hdg_ctx* out);

hdg_status hdg_query_sizes(hdg_ctx ctx, hdg_sizes* out);

/* Per-macro offsets (host arrays of n_macros + 1 entries, either may be
 * NULL): u_off[i] = first entry of macro i in u (q: dim * u_off[i]);
 * b_off[i] = first entry of macro i's boundary trace vector in the
 * concatenation of all macros' local trace vectors (n_b per macro). */
hdg_status hdg_macro_offsets(hdg_ctx ctx, long long* u_off, long long* b_off);

/* face_off (host, n_faces + 1 entries): first entry of each face in uhat. */
hdg_status hdg_face_offsets(hdg_ctx ctx, long long* face_off);

/* Node coordinates for building inputs: macro nodes [macro][node][dim] and
 * trace nodes [face][facenode][dim], host arrays of n_u_tot/(dim+2)*dim and
 * n_glob/(dim+2)*dim doubles (either may be NULL). */
hdg_status hdg_node_coords(hdg_ctx ctx, double* macro_xyz_host, double* face_xyz_host);

/* Caller-owned device workspace of at least workspace_bytes (256-byte
 * aligned).  Must be bound before hdg_linearize_stage. */
hdg_status hdg_bind_workspace(hdg_ctx ctx, void* dev_ptr, size_t bytes);

/* Chunked condensation, for meshes whose augmented macro matrices
 * (n_u + n_b)^2 per macro do not fit in device memory at once (the local
 * problems are independent per macro, Sec. 3.3, so they can be processed in
 * groups).  macros_per_chunk > 0 and below n_macros: hdg_condense forms and
 * eliminates consecutive ranges of that many macros (the first range takes
 * the remainder of n_macros / macros_per_chunk) through one buffer and
 * keeps only the condensed blocks A-hat^{T_i} (compact, in the condensation
 * precision) and b-hat^{T_i}; hdg_local_backsolve forms and factors each
 * range's S again (the S rows only, with the right-hand side f + C duhat of
 * eq. Csc4a folded into one column: the LU of S carries that column alone),
 * except the ranges whose factors it still has (the last range condensed,
 * left in W, see hdg_set_chunk_buffers, and the factor store, see
 * hdg_set_factor_store).  0 (default) or >= n_macros: everything at once.
 * Re-plans the workspace: call hdg_query_sizes and hdg_bind_workspace again
 * afterwards (any bound workspace and learned network are released).
 * With chunking, an FP32 inner operator (hdg_krylov_opts.inner_prec) needs
 * an FP32 condensation (HDG_EUNSUPPORTED otherwise), and
 * hdg_get_formed forms only the macro's chunk.  HDG_EINVAL when the number
 * of chunks times the number of macro classes exceeds 4095. */
hdg_status hdg_set_chunking(hdg_ctx ctx, int macros_per_chunk);

/* Chunk slots of the W buffer under chunked condensation: 1 (default) or 2.
 * With 2, W holds two chunks (chunk j in slot j % 2, so twice the W bytes for
 * the same macros_per_chunk): hdg_condense forms chunk j + 1 on a second
 * stream of the library's while chunk j is eliminated on the library's
 * stream (the local problems of different macros are independent, Sec. 3.3);
 * hdg_local_backsolve does the same for the chunks it forms again.  With
 * either setting, hdg_local_backsolve recovers the chunks whose eliminations
 * W still holds from the last hdg_condense (one per slot) from those factors,
 * when no call that writes W (hdg_linearize_stage, hdg_autotune,
 * hdg_get_formed, hdg_condense_first_layer, a recovery that formed chunks
 * again) came in between.  No effect without chunking.  Re-plans the
 * workspace like hdg_set_chunking.  HDG_EINVAL for other values. */
hdg_status hdg_set_chunk_buffers(hdg_ctx ctx, int n_buffers);

/* Factor store for the recovery under chunked condensation: hdg_condense
 * copies the LU factors of S (P S = L U of eq. ASC2, the top-left n_u x n_u
 * of each eliminated matrix, 16 x 64 tiles with ld = n_u rounded up to 64)
 * of the macros of the leading whole chunks that fit in n_macros (never the
 * last chunk of a W slot, which stays in W) into workspace memory of type
 * prec (HDG_FP64: 8, HDG_FP32: 4 bytes per entry).  hdg_local_backsolve then
 * solves S dU = r for those macros from the store, with r the residual of
 * the u-rows of eq. C44 in FP64 (dQ from eq. Csc4b): once for FP64 factors
 * of an FP64 condensation, three FP64 refinement sweeps for FP32 factors
 * (or an FP32 condensation), instead of forming and factoring their S again.
 * The pivots are the condensation's.  hdg_linearize_stage, hdg_autotune,
 * hdg_condense_first_layer and any re-planning invalidate the store until
 * the next hdg_condense.  Re-plans the workspace like hdg_set_chunking.
 * HDG_EINVAL for n_macros < 0, HDG_EUNSUPPORTED for other precisions. */
hdg_status hdg_set_factor_store(hdg_ctx ctx, int n_macros, hdg_prec prec);
/* Macros the factor store holds under the current plan (whole chunks). */
hdg_status hdg_factor_store_macros(hdg_ctx ctx, int* n_stored);

/* Progress lines for long runs (for instance under a profiler that
 * serialises every kernel): with on != 0, hdg_condense and
 * hdg_local_backsolve wait for the library's stream after each chunk and
 * print "[hdg] <phase> <i> of <n> done" on stderr.  Off by default. */
hdg_status hdg_set_progress(hdg_ctx ctx, int on);

/* Autotuner of the batched elimination of hdg_condense: for every macro
 * class (one per macro shape) and the given condensation precision, times
 * the class's elimination (HIP events on the context's stream, after one
 * untimed trial) for each candidate launch shape -- 8, 16, 32, 64, 128 or
 * 256 sixteen-row tiles per workgroup of the trailing update with the 512-thread
 * panel factorisation, then the 1024-thread panel and tournament pivoting
 * with the best of those, then the factorisation of the next pair of column
 * blocks on a second stream beside the trailing update -- on the current
 * linearisation, and keeps the fastest (another panel and the second stream
 * only when they gain more than 2%, the spread of single timings).
 * cache_path (host string, may be NULL): text file of earlier choices, one
 * line per (GPU architecture, HIP runtime version, precision, class shape,
 * batch size); classes found there are not timed, new choices are appended.
 * n_timed (host, may be NULL) receives the number of classes timed.
 * Needs a bound workspace and a prior hdg_linearize_stage; the trials
 * overwrite the condensed blocks, so hdg_condense must follow.  The choices
 * change launch shapes and, with tournament pivoting, the pivot order; the
 * results differ by rounding only. */
hdg_status hdg_autotune(hdg_ctx ctx, hdg_prec prec, const char* cache_path, int* n_timed);

/* Number of macro classes (distinct macro shapes) of the mesh. */
hdg_status hdg_class_count(hdg_ctx ctx, int* n_classes);

/* Launch shape in use for class macro_class (0 .. n_classes - 1) and the
 * given precision: tiles per workgroup of the trailing update (default 32),
 * the panel kind (default 2) and the look-ahead-stream flag (default 0);
 * host pointers, each may be NULL.  Panel kinds: 0 partial pivoting in one
 * 512-thread workgroup per matrix (LAPACK's pivot order), 1 the same with
 * 1024 threads, 2 tournament pivoting (the block's pivot rows chosen by
 * rounds of partial pivoting over groups of 256 rows, then L21 = A21 U11^-1
 * on MFMA). */
hdg_status hdg_get_tuning(hdg_ctx ctx, int macro_class, hdg_prec prec, int* tpw, int* panel, int* lookahead);

/* Sets the launch shape of a class by hand (tpw: multiple of 4 in [4, 256];
 * panel 0, 1 or 2; lookahead 0 or 1); HDG_EINVAL otherwise.  Results change
 * only by rounding. */
hdg_status hdg_set_tuning(hdg_ctx ctx, int macro_class, hdg_prec prec, int tpw, int panel, int lookahead);

/* Linearise eq. (C242) at (q, u, uhat): residuals R_Q, R_U, R_Uhat and the
 * Jacobian blocks of eq. (C312) of every macro, kept in the workspace.
 * w: stage history with the discrete time derivative (d_ii u + w) / dt
 * (w = sum_{j<i} d_ij (u^{n,j} - u^n) - d_ii u^n), layout of u; NULL = 0.
 * dt = INFINITY: steady (no time term).  dtau: pseudo-time step of the
 * continuation (adds M / dtau to A_uu); INFINITY = off.
 * norms_host (may be NULL): ||R_Q||_2, ||R_U||_2, ||R_Uhat||_2 (synchronises). */
hdg_status hdg_linearize_stage(hdg_ctx ctx, const double* q, const double* u, const double* uhat,
                               const double* w, double dt, double d_ii, double dtau,
                               double norms_host[3]);

/* Second-layer static condensation (eq. AP12, ASC2a/b): per macro the Schur
 * complement S = A_uu - A_uq A_qq^{-1} A_qu is LU-factored with partial
 * pivoting and the condensed blocks A-hat^{T_i} and right-hand sides
 * b-hat^{T_i} are formed; bhat (device, n_glob) receives the assembled b-hat
 * of eq. (C44).  Also factors the face blocks of A_uhat-uhat used by the
 * preconditioner.
 * prec = HDG_FP64: formation and elimination in FP64 (FP64 MFMA).
 * prec = HDG_FP32: the augmented matrices are formed with FP32 sums (g of
 *   eq. ASC2b in FP64, kept outside the matrix) and stored in FP32 and
 *   eliminated with FP32 arithmetic (FP32 MFMA); the
 *   condensed blocks, b-hat and the operator of hdg_apply_global then carry
 *   FP32 rounding (vectors and sums stay FP64; hdg_local_backsolve refines
 *   its S-solves to FP64).  A Newton iteration whose residuals are
 *   evaluated in FP64 (hdg_linearize_stage) refines the result back to the
 *   FP64 level.  The precision stays in effect until the next hdg_condense.
 * prec = HDG_BF16: as HDG_FP32 (FP32 storage, formation and panel
 *   factorisations) but the trailing updates of the elimination (the Schur
 *   products L21 U12, which carry nearly all the flops) take BF16 operands
 *   (rounded to nearest even) with FP32 accumulation on the BF16 MFMA units:
 *   the condensed blocks carry errors of about 1e-3 to 1e-2 relative, which
 *   the Newton iteration refines at a correspondingly slower rate; the
 *   recovery's FP64 refinement takes more sweeps.
 * The face blocks of the preconditioner are always FP64.
 * Returns HDG_ESINGULAR (message names the macro) on a zero pivot. */
hdg_status hdg_condense(hdg_ctx ctx, hdg_prec prec, double* bhat);

/* First-layer (standard) static condensation (Sec. 3.2, eq. C46/C47), for
 * comparison with hdg_condense: (q, u) of every macro are eliminated
 * together -- an LU with partial pivoting of the local matrix
 * [[A_qq, A_qu], [A_uq, A_uu]] of order n_q + n_u -- giving the same
 * A-hat^{T_i} and b-hat^{T_i} (to rounding) and the same assembled bhat
 * (device, n_glob); FP64.  Afterwards hdg_apply_global, hdg_fgmres_solve
 * and hdg_local_backsolve (which forms and factors S again per chunk) work
 * as after hdg_condense(HDG_FP64).  Needs chunking (hdg_set_chunking; the W
 * buffer holds as many first-layer matrices at a time as fit) and a mesh of
 * one macro shape, and n_q + n_u <= 12288 with a row of at most 150 KiB
 * in FP64 (HDG_EUNSUPPORTED otherwise); HDG_ENOMEM when the W
 * buffer cannot hold one first-layer matrix; HDG_ESINGULAR on a zero
 * pivot. */
hdg_status hdg_condense_first_layer(hdg_ctx ctx, double* bhat);

/* Nested hybridisation inside a macro: a third static-condensation layer,
 * the alternative local structure in which every element is hybridised on
 * its own (u, q discontinuous between elements, a trace on every element
 * face; the paper's Sec. 2.2 patches instead keep u, q continuous inside a
 * macro).  On a mesh of one element per macro (all macros of one shape,
 * m = 1 on every axis), the elements are grouped into blocks of block_m
 * elements per axis (block (g0, g1[, g2]) = g0 + n0 (g1 + n1 g2), element
 * s belongs to block s_k / block_m per axis).  Each block assembles the
 * element blocks A-hat^{T_e}, b-hat^{T_e} of the last FP64 hdg_condense
 * (eq. C44 pieces) over the faces of its elements and eliminates the traces
 * of the faces inside the block, as eq. ASC2 eliminates u:
 *   A-hat^G = A_BB - A_BI A_II^{-1} A_IB,  b-hat^G = b_B - A_BI A_II^{-1} b_I,
 * which leaves a system on the block skeleton (faces between blocks and on
 * the domain boundary), assembled like eq. C44.  Block-local trace order:
 * the block's internal faces in increasing face id, then its boundary faces
 * likewise, each face's unknowns in their global order (hdg_face_offsets).
 *
 * hdg_nested_dims: number of blocks and, per block, the internal-face and
 * boundary-face trace unknowns (host pointers, each may be NULL).
 * hdg_condense_nested: ahat (device, n_blocks x n_B x n_B row-major) and bhat
 * (device, n_blocks x n_B) receive A-hat^G and b-hat^G on each block's
 * boundary faces; synchronises.  Needs a bound workspace and an FP64
 * hdg_condense of the current linearisation (HDG_EINVAL otherwise; a later
 * linearisation, autotune or first-layer condensation invalidates it).
 * HDG_EINVAL when the element count of an axis is not a multiple of
 * block_m; HDG_EUNSUPPORTED for other meshes (several macro shapes, m > 1,
 * a periodic axis of one element, blocks of unequal face counts, more than
 * 12288 internal-face unknowns per block); HDG_ENOMEM when its buffers do
 * not fit; HDG_ESINGULAR on a zero pivot of A_II.  The block structure and
 * its device buffers (n_blocks tiled matrices of order n_I + n_B) are
 * allocated on the first call for a block size and kept until the block
 * size changes or hdg_destroy. */
hdg_status hdg_nested_dims(hdg_ctx ctx, int block_m, int* n_blocks, int* n_internal, int* n_boundary);
hdg_status hdg_condense_nested(hdg_ctx ctx, int block_m, double* ahat, double* bhat);

/* Solve of the nested (block-skeleton) system of the last hdg_condense_nested
 * with this block size (HDG_EINVAL otherwise): FGMRES as in hdg_fgmres_solve
 * (sec. 4.2; options o as there, but host-controlled FP64 steps only:
 * graph_steps, use_learned and harvest_max 0, inner_prec HDG_FP64, else
 * HDG_EUNSUPPORTED) from a zero start, the inner GMRES preconditioned by the
 * diagonal of the skeleton operator, applied matrix-free as
 * sum_G P_G^T A-hat^G P_G (deterministic owner sums).  Then the traces of
 * every block's internal faces, x_I = A_II^{-1} (b_I - A_IB x_B), from the
 * factors the elimination left in the block matrices.  x_full (device,
 * n_glob) receives the whole element-trace increment in the layout of
 * hdg_face_offsets; hdg_local_backsolve turns it into dq, du as after
 * hdg_fgmres_solve.  st (host, may be NULL) as for hdg_fgmres_solve.
 * HDG_ENOCONV when max_outer is reached (x_full then holds the recovery of
 * the last iterate). */
hdg_status hdg_nested_solve(hdg_ctx ctx, int block_m, double* x_full, const hdg_krylov_opts* o,
                            hdg_krylov_stats* st);

/* Flow diagnostics of the Taylor-Green study (Sec. 5.3, eq. C5321) for the
 * state (q, u) (device, layouts as in hdg_linearize_stage), in the
 * library's units (rho_inf = c_inf = mu = 1, mu_eff = mu / Re_c):
 *   out_host[0] = E_k = (1/|Omega|) int 1/2 rho |v|^2,
 *   out_host[1] = eps = 2 mu_eff / |Omega| int rho |omega|^2 / 2, omega = curl v
 *                 (2D: the scalar d_x v_y - d_y v_x), the velocity gradient
 *                 from q by the chain rule d_k v_j = (q_k[m_j] - v_j q_k[rho]) / rho,
 *   out_host[2] = |Omega|,
 * integrated with the element quadrature; deterministic (fixed summation
 * order).  Uses the workspace's reduction buffer; synchronises the stream.
 * A state with rho <= 0 gives non-finite values (no error).
 * HDG_EINVAL on null pointers, HDG_ENOMEM without a workspace. */
hdg_status hdg_flow_diagnostics(hdg_ctx ctx, const double* q, const double* u, double out_host[3]);

/* hdg_flow_diagnostics for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, bit for bit, but the
 * per-workgroup partial sums and the three results live in a static device
 * array of the library (4 + 3 * 65536 doubles, about 1.5 MiB per device,
 * held until the process ends) instead of the workspace, so no workspace
 * needs to be bound and the call allocates nothing (the host result goes
 * through a pinned buffer made at set-up).  The array holds a fixed number of
 * partial sums whatever the mesh size (larger meshes fold more elements into
 * each); HDG_EINVAL if a mesh would need more.  Every call on one GPU shares
 * that GPU's array and overwrites it before reading it: calls that overlap
 * on one GPU (several threads or streams) race.  Synchronises the stream. */
hdg_status hdg_flow_diagnostics_noalloc(hdg_ctx ctx, const double* q, const double* u, double out_host[3]);

/* y = A-hat x = sum_i P_i^T A-hat^{T_i} P_i x (Algorithm 2 with the condensed
 * blocks formed by hdg_condense, in the precision of that call; sums in
 * FP64); x, y device, n_glob, must not alias. */
hdg_status hdg_apply_global(hdg_ctx ctx, const double* x, double* y);

/* Solve A-hat x = b with the options above (Sec. 4.2).  x: initial guess on
 * input, solution on output.  Returns HDG_ENOCONV (x = last iterate, stats
 * filled) when max_outer is reached. */
hdg_status hdg_fgmres_solve(hdg_ctx ctx, const double* b, double* x, const hdg_krylov_opts* opts,
                            hdg_krylov_stats* stats_host);

/* Local recovery (eq. Csc4a then Csc4b): dU and dQ of every macro from the
 * trace increment duhat (device, n_glob).  dq, du device, layouts of q, u.
 * After an FP32 condensation the S-solve is refined in FP64: two sweeps of
 * dU += S_32^{-1} r with r = -(R_U + A_uq dQ + A_uu dU + A_u,uh duhat), the
 * FP64 residual of the u-rows of the Newton system (eq. C312) from the
 * linearisation's blocks, so dU and dQ are FP64-accurate.  Chunked, the
 * macros of the factor store are solved the same way from dU = 0 (see
 * hdg_set_factor_store).  The residual uses the Krylov vectors of the
 * workspace as scratch (HDG_EDEVICE if n_u_tot exceeds them). */
hdg_status hdg_local_backsolve(hdg_ctx ctx, const double* duhat, double* dq, double* du);

/* y += a x on n doubles (device): the Newton update. */
hdg_status hdg_axpy(hdg_ctx ctx, size_t n, double a, const double* x, double* y);

/* Plain preconditioner stage on its own: z = inner_its steps of GMRES (zero
 * start) on A-hat left-preconditioned by the inverse face blocks of
 * A_uhat-uhat (Sec. 4.2), plus the learned coarse correction if use_learned
 * and a network is bound.  v, z device, n_glob, must not alias.  Valid after
 * hdg_condense. */
hdg_status hdg_precond_apply(hdg_ctx ctx, const double* v, double* z, int inner_its, hdg_prec inner_prec,
                             int use_learned);

/* ---- learned coarse correction --------------------------------------------
 * Not part of the paper: a stage that FGMRES's flexibility (Sec. 4.2)
 * admits.  Coarse space: per macro face and component, the multilinear
 * functions of the tangential face coordinates (scaled to [0, 1] over the
 * face); 2d n_s 2^(d-1) coefficients per macro (120 in 3D), ordered
 * [local face][component][function] with functions (1-s)(1-t), s(1-t),
 * (1-s)t, st (3D; 1-s, s in 2D). */

/* Number of coarse coefficients per macro. */
hdg_status hdg_coarse_size(hdg_ctx ctx, int* n_features);

/* X [n_macros][n_features] (device, FP32) = discrete L2 projection of the
 * face fields of v (device, n_glob) onto the coarse functions, with the
 * composite Gauss-Lobatto rule of the face nodes as inner product. */
hdg_status hdg_coarse_restrict(hdg_ctx ctx, const double* v, float* X);

/* z += alpha * (coarse functions with coefficients Y evaluated at the face
 * nodes), each face taking the mean over the macros that own it. */
hdg_status hdg_coarse_prolong(hdg_ctx ctx, const float* Y, double alpha, double* z);

/* Xe [n_macros][(1 + 2d) n_features] (device, FP32; X and Xe must not
 * overlap) = per macro its own row of X, then the rows of the macros across
 * its local faces 0 .. 2d-1 (zeros across a face on the domain boundary):
 * the input of a network that sees the coarse state of the face
 * neighbours. */
hdg_status hdg_coarse_neighbours(hdg_ctx ctx, const float* X, float* Xe);

/* Two-layer network y = ||x|| (W2 tanh(W1 x / ||x|| + b1) + b2) (y = 0 for
 * x = 0).  All arrays are caller-owned device memory in FP32. */
typedef struct {
  int n_in, n_hidden, n_out;  /* n_hidden <= 512 for hdg_learned_bind */
  int max_batch;              /* rows per call of the training entry points */
  float* params;  /* W1 [n_hidden][n_in], b1 [n_hidden], W2 [n_out][n_hidden], b2 [n_out] */
  float* grads;   /* layout of params (written by hdg_mlp_loss_grad) */
  float* adam_m;  /* layout of params, zero before the first hdg_mlp_adam */
  float* adam_v;  /* layout of params, zero before the first hdg_mlp_adam */
  float* work;    /* hdg_mlp_work_floats() floats of scratch */
} hdg_mlp;

size_t hdg_mlp_param_count(int n_in, int n_hidden, int n_out);
size_t hdg_mlp_work_floats(int n_in, int n_hidden, int n_out, int max_batch);

/* Y [batch][n_out] = network applied to the rows idx[0..batch) of X (idx
 * device, NULL = rows 0..batch-1); FP32.  batch <= max_batch. */
hdg_status hdg_mlp_forward(hdg_ctx ctx, const hdg_mlp* net, const float* X, const int* idx, int batch, float* Y);

/* Mean squared error over the batch and the outputs between the network
 * before rescaling and T / ||x|| (normalised units), and its gradient with
 * respect to params (into net->grads).  loss_dev (device, may be NULL)
 * receives the loss. */
hdg_status hdg_mlp_loss_grad(hdg_ctx ctx, const hdg_mlp* net, const float* X, const float* T, const int* idx,
                             int batch, float* loss_dev);

/* One Adam step (Kingma and Ba) on params with net->grads; step counts from 1. */
hdg_status hdg_mlp_adam(hdg_ctx ctx, const hdg_mlp* net, float lr, float beta1, float beta2, float eps, int step);

/* Copy the network's parameters to BF16 inside the context for use by the
 * preconditioner (n_out = hdg_coarse_size; n_in = hdg_coarse_size, or
 * (1 + 2d) hdg_coarse_size for a network fed by hdg_coarse_neighbours;
 * n_hidden <= 512); NULL unbinds.  The copy is taken when the call's work
 * runs on the stream. */
hdg_status hdg_learned_bind(hdg_ctx ctx, const hdg_mlp* net);

hdg_status hdg_destroy(hdg_ctx ctx);
const char* hdg_status_string(hdg_status s);
const char* hdg_last_error(hdg_ctx ctx);

/* Inspection (tests): copy macro `macro`'s condensed block A-hat^{T_i}
 * (n_b x n_b row-major, n_b of that macro) and b-hat^{T_i} (n_b) to host
 * memory (synchronises).
 * Valid after hdg_condense. */
hdg_status hdg_get_condensed(hdg_ctx ctx, size_t macro, double* ahat_host, double* bhat_host);

/* Inspection (tests): run only the formation step of hdg_condense and copy
 * the augmented matrix [[S, -C, f], [D, E, g]] of macro `macro` to host
 * ((n_u + n_b) x (n_u + n_b + 1) row-major, sizes of that macro), with C = -A_u,uhat + A_uq
 * A_qq^{-1} A_q,uhat, f = A_uq A_qq^{-1} R_Q - R_U, D = A_uhat,u - A_uhat,q
 * A_qq^{-1} A_qu, E = A_uhat,uhat - A_uhat,q A_qq^{-1} A_q,uhat, g = -R_Uhat +
 * A_uhat,q A_qq^{-1} R_Q (eq. ASC2).  Valid after hdg_linearize_stage. */
hdg_status hdg_get_formed(hdg_ctx ctx, size_t macro, double* w_host);

/* Inspection (tests): residual vectors of the last linearisation (device
 * outputs, layouts of q, u, uhat; R_Uhat summed over both sides). */
hdg_status hdg_get_residuals(hdg_ctx ctx, double* rq, double* ru, double* rb);

#ifdef __cplusplus
}
#endif
#endif

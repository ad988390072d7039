// Host-side context of libhdg.so: mesh topology, reference tables of the
// macro shape, workspace layout.  Internal.
#pragma once
#include "internal.h"
#include <algorithm>
#include <array>
#include <map>
#include <memory>

struct NestedPlan;  // block structure and buffers of the nested (third-layer) condensation, k_nested.hip

struct HostClass {
  int dim, p, nq, ns;
  int m[3], n1[3];
  int N, E, A, Q, T, Fq, n_u, n_q, n_b, n_sub, nmax1;
  double h[3];
  int nf_nodes[HDG_MAXF], nf_off[HDG_MAXF];
  std::vector<double> Phi, dPhi, W, Tvol, Mel, Psi, WF, C1D, Minv1D, M1D, B1D;
  int cq = 0, cF = 0, cmaxf = 0;
  std::vector<double> cR, cPhi;
  // tiled augmented matrix
  int ldw = 0, n_rows = 0, n_cols = 0;
  long long wstride = 0;
  LuTune tune[2];  // elimination launch choices for FP64 and FP32 storage
  std::vector<int> fnode, finv, elem_nodes, elem_sub, sub_elem, sub_lf, sub_tid, node_ne, node_e, node_a,
      tn_cnt, tn_sub, tn_t, tn_base;
};

struct HostMesh {
  int dim, ns, p;
  int n_elem[3], n_seg[3], periodic[3];
  double lo[3], hi[3], h[3];
  std::vector<int> seg_len[3], seg_start[3];
  int n_macros, n_faces;
  long long n_glob;
  std::vector<int> macro_face, macro_bnd, face_axis, face_minus, face_plus, face_ndof, face_nodes;
  std::vector<long long> face_off;
  std::vector<std::array<int, 3>> face_grid;
  // macro classes (distinct m per axis) and per-macro offsets
  int n_classes = 0;
  std::vector<std::array<int, 3>> class_m;        // m per axis of each class
  std::vector<int> macro_class;                   // [n_macros]
  std::vector<long long> u_off, b_off, el_off, sub_off, row_off, a32_off;  // [n_macros + 1]
  std::vector<int> elem_macro;
  std::vector<long long> w_off, ipiv_off;         // [n_macros], grouped by class
  std::vector<long long> class_w_base, class_ipiv_base;
  std::vector<int> class_count, class_first;      // macros per class; first macro of the class
  // face-preconditioner blocks stored grouped by face size: slot of each face,
  // and per distinct size (trace unknowns, first slot, count)
  std::vector<int> face_slot;
  std::vector<std::array<int, 3>> face_groups;
  // chunked condensation: the macros are condensed in consecutive ranges
  // [chunk_first[j], chunk_first[j + 1]) through W, which holds chunk_buffers
  // slots each sized for the largest range (chunk j in slot j % chunk_buffers);
  // w_off is then relative to W.  Per (chunk, class): offset of the class's
  // matrices in W, their count and the rank (within the class) of the first
  // of them.
  int chunk_macros = 0;                  // requested macros per chunk (0: all at once)
  int chunk_buffers = 1;                 // chunk slots in W (2: the next chunk is formed beside this one's elimination)
  // factor store: copies of the LU factors of S (the top-left n_u x n_u of the
  // eliminated W, tiled 16 x 64 with ld = n_u rounded up to 64) of the macros
  // of the leading chunks [0, store_chunks), in store_prec (0 FP64, 1 FP32),
  // at st_off[macro] (-1: not stored) in elements of that type
  int store_macros = 0;                  // requested number of macros
  int store_prec = 1;
  int store_chunks = 0;
  std::vector<long long> st_off;         // [n_macros]
  std::vector<int> chunk_first;          // [n_chunks + 1]
  std::vector<long long> chunk_class_w;  // [n_chunks * n_classes]
  std::vector<int> chunk_class_cnt, chunk_class_rank0;
  int n_chunks() const { return (int)chunk_first.size() - 1; }
  bool chunked() const { return n_chunks() > 1; }
  int slots() const { return chunked() ? std::min(chunk_buffers, n_chunks()) : 1; }
};

struct Workspace {
  char* base = nullptr;
  size_t bytes = 0;
  double* Kq = nullptr;     // pointwise flux-Jacobian scratch, [elements][Kstride]
  double* AUU = nullptr;    // [elements][nsA][nsA]
  double* AUQ = nullptr;    // [elements][nsA][d nsA]
  double* RUe = nullptr;    // [elements][nsA]
  double* RQe = nullptr;    // [elements][d nsA]
  double* SUB = nullptr;    // [macros * n_sub][sub_stride]
  double* RU = nullptr;     // [n_u_tot]
  double* RQ = nullptr;     // [n_q_tot]
  double* RQt = nullptr;    // [n_q_tot]  M^{-1} R_Q per direction and component
  double* RBloc = nullptr;  // [macros][n_b] per-macro trace residual
  double* RBglob = nullptr; // [n_glob]
  double* gloc = nullptr;   // [macros][n_b] g of eq. ASC2b in FP64 (FP32 condensation keeps it out of W)
  double* Wm = nullptr;     // [macros][n_rows][ldw] augmented matrices (FP64, or FP32 in the first half)
  int* ipiv = nullptr;      // [macros][n_u]
  double* FW = nullptr;     // [faces][2 nf][ldf] face preconditioner
  int* fpiv = nullptr;      // [faces][nf]
  float* A32 = nullptr;     // [macros][n_b][n_b] FP32 copy of A-hat (inner operator)
  unsigned short* A16 = nullptr;  // [macros][n_b][n_b] BF16 copy of A-hat (inner operator)
  double* ypart = nullptr;  // [macros][n_b]
  double* kry = nullptr;    // Krylov vectors
  double* red = nullptr;    // reduction scratch
  double* small = nullptr;  // small device scalars
  double* Uinv = nullptr;   // [max(macros, faces)][64][64] block inverses of the elimination
  float* lrn = nullptr;     // learned stage: X, Y [macros][cF] each, then the BF16 network
  double* kctl = nullptr;   // device-resident Krylov control block (Hessenbergs, rotations, scalars)
  double* supg = nullptr;   // SUPG products of a chunk of elements (only with SUPG on)
  // chunked condensation only (Wm then holds one chunk and shares its memory with Kq)
  double* Ac = nullptr;     // [macros][n_b][n_b] compact A-hat (FP64, or FP32 in the first half)
  double* bloc = nullptr;   // [macros][n_b] b-hat^{T_i}
  double* Fst = nullptr;    // factor store (FP64 or FP32 elements at HostMesh::st_off)
};

struct HdgContext {
  HostMesh hm;
  HostClass hc;               // class 0 (degree-dependent tables are the same for every class)
  ClassDev cd{};              // device view of class 0
  std::vector<HostClass> hcs; // every class
  std::vector<ClassDev> cds;  // device views of every class (uploaded as MeshDev::cls)
  PhysDev ph{};
  MeshDev md{};
  hipStream_t stream = nullptr;
  int device = -1;                // HIP device current at set-up (the stream's device)
  std::vector<void*> dev_allocs;  // small tables owned by the context
  Workspace ws;
  bool ws_bound = false;
  // sizes
  long long n_u_tot = 0, n_q_tot = 0;
  int n_rows = 0, n_cols = 0, ldw = 0;  // augmented matrix
  long long wstride = 0;                // doubles per tiled macro matrix
  long long fstride = 0;                // doubles per tiled face-preconditioner block
  int nsA = 0, dnsA = 0, sub_stride = 0, Kstride = 0;
  int nf_max = 0, ldf = 0;
  int kry_restart_max = 64, kry_inner_max = 16;
  size_t need_bytes = 0;
  size_t wm_bytes = 0;  // size of the W buffer
  // offsets of the sub-face block pieces
  int off_AUB = 0, off_ABU = 0, off_ABQ = 0, off_ABB = 0, off_RB = 0;
  bool have_a32 = false;
  bool have_a16 = false;
  bool linearized = false;  // element blocks hold a linearisation
  int cond_prec = 0;  // element type of the condensed matrices in W: 0 FP64, 1 FP32
  bool condensed64 = false;  // the element blocks of the last FP64 hdg_condense are in place
  // chunked: the chunks whose condensations W still holds (-1: none), the
  // last ones condensed, one per slot
  int w_res[2] = {-1, -1};
  void forget_w() { w_res[0] = w_res[1] = -1; }
  bool store_valid = false;             // the factor store holds the factors of the last hdg_condense
  bool progress = false;                // a line on stderr per finished chunk (hdg_set_progress)
  const long long* st_off_dev = nullptr; // device copy of HostMesh::st_off
  std::shared_ptr<NestedPlan> nested;  // nested condensation for one block size (built on first use)
  int nested_m = 0;                    // its block size
  bool bf16_update = false;  // the last condensation took BF16 operands in its trailing updates
  long long supg_chunk = 0;  // elements per SUPG product batch
  // learned coarse correction
  bool lrn_bound = false;
  int lrn_hidden = 0;
  int lrn_in = 0;  // network inputs: cF (own macro) or (1 + 2d) cF (with the face neighbours)
  // captured FGMRES steps: key (first step, steps, restart, inner its, inner prec,
  // condensed prec, learned, FP32 copy present) -> executable graph
  std::map<std::array<int, 8>, hipGraphExec_t> graphs;
  hipStream_t cap_stream = nullptr;  // private stream used only for capture
  // streams on which the per-class eliminations run concurrently (created on
  // first use when the mesh has several macro classes), with fork/join events
  std::vector<hipStream_t> lu_streams;
  std::vector<hipEvent_t> lu_events;
  // per class slot: the look-ahead panel stream and its two hand-off events
  std::vector<hipStream_t> lu_pstreams;
  std::vector<hipEvent_t> lu_pevents;
  // two chunk slots: the formation stream and its events (start, formed per
  // slot, slot free per slot), created on first use
  hipStream_t form_stream = nullptr;
  hipEvent_t form_events[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  std::string last_error;
};

struct HdgMeshIn {
  int dim;
  int n_elem[3];
  double lo[3], hi[3];
  int periodic[3];
  int n_seg[3];
  const int* seg_len[3];
  int p;
};

// k_nested.hip
std::string nested_plan(HdgContext& c, int M, std::shared_ptr<NestedPlan>& out);
hipError_t launch_condense_nested(HdgContext& c, NestedPlan& P, double* ahat, double* bhat, int* singular);
void nested_dims(const NestedPlan& P, int* n_blocks, int* n_internal, int* n_boundary);
hipError_t launch_nested_apply(HdgContext& c, NestedPlan& P, const double* x, double* y);
hipError_t launch_nested_jacobi(HdgContext& c, NestedPlan& P, const double* v, double* z);
hipError_t launch_nested_recover(HdgContext& c, NestedPlan& P, const double* xskel, double* xfull);
long long nested_skeleton_size(const NestedPlan& P);
bool nested_condensed(const NestedPlan& P);
double* nested_rhs(NestedPlan& P);
double* nested_xskel(NestedPlan& P);

// host_setup.cpp
bool build_mesh(const HdgMeshIn& in, HostMesh& hm, std::string& err);
void build_class(const HostMesh& hm, HostClass& hc, const std::array<int, 3>& m);
void plan_workspace(HdgContext& c);
void upload_tables(HdgContext& c);
void upload_w_offsets(HdgContext& c);
void node_coords(const HdgContext& c, double* macro_xyz, double* face_xyz);


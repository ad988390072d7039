"""Thin ctypes binding of libhdg.so (include/hdg.h), same call names.

Argument marshalling only: device arrays are passed as torch CUDA tensors
(their data pointers), work is queued on torch's current stream.  Every step
of the path runs in the library's HIP kernels; there is no fallback, and a
missing library raises at import of this module's Context.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdg.so")

HDG_FP64, HDG_FP32, HDG_BF16 = 0, 1, 2
_STATUS = {0: "HDG_OK", 1: "HDG_EINVAL", 2: "HDG_ENOMEM", 3: "HDG_EDEVICE", 4: "HDG_ESINGULAR",
           5: "HDG_ENOCONV", 6: "HDG_EBREAKDOWN", 7: "HDG_ENAN", 8: "HDG_EUNSUPPORTED"}


class HdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class _MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_elem", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("periodic", ctypes.c_int * 3), ("n_seg", ctypes.c_int * 3),
                ("seg_len", ctypes.POINTER(ctypes.c_int) * 3), ("p", ctypes.c_int)]


class _Phys(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("Re", ctypes.c_double),
                ("Mach", ctypes.c_double), ("supg", ctypes.c_int), ("bc_state_host", ctypes.POINTER(ctypes.c_double))]


class _Sizes(ctypes.Structure):
    _fields_ = [("n_macros", ctypes.c_size_t), ("n_glob", ctypes.c_size_t), ("n_u_tot", ctypes.c_size_t),
                ("n_q_tot", ctypes.c_size_t), ("n_u_macro", ctypes.c_size_t), ("n_b_macro", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t), ("n_faces", ctypes.c_size_t)]


class KrylovOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("restart", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("inner_its", ctypes.c_int), ("inner_prec", ctypes.c_int),
                ("use_learned", ctypes.c_int), ("no_fallback", ctypes.c_int), ("harvest", ctypes.c_void_p),
                ("harvest_max", ctypes.c_int), ("graph_steps", ctypes.c_int)]


class KrylovStats(ctypes.Structure):
    _fields_ = [("outer_its", ctypes.c_int), ("inner_its_total", ctypes.c_int), ("res0", ctypes.c_double),
                ("res_final", ctypes.c_double), ("ms", ctypes.c_double), ("fallbacks", ctypes.c_int),
                ("harvested", ctypes.c_int)]


class Mlp(ctypes.Structure):
    """hdg_mlp: shape and device pointers of a two-layer network."""
    _fields_ = [("n_in", ctypes.c_int), ("n_hidden", ctypes.c_int), ("n_out", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("params", ctypes.c_void_p), ("grads", ctypes.c_void_p),
                ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p), ("work", ctypes.c_void_p)]


EXPORTS = ["hdg_setup_mesh", "hdg_query_sizes", "hdg_macro_offsets", "hdg_face_offsets", "hdg_node_coords", "hdg_bind_workspace", "hdg_linearize_stage",
           "hdg_condense", "hdg_apply_global", "hdg_fgmres_solve", "hdg_local_backsolve", "hdg_axpy",
           "hdg_destroy", "hdg_status_string", "hdg_last_error", "hdg_get_condensed", "hdg_get_formed",
           "hdg_get_residuals", "hdg_precond_apply", "hdg_coarse_size", "hdg_coarse_restrict", "hdg_coarse_neighbours",
           "hdg_coarse_prolong", "hdg_mlp_param_count", "hdg_mlp_work_floats", "hdg_mlp_forward",
           "hdg_mlp_loss_grad", "hdg_mlp_adam", "hdg_learned_bind", "hdg_set_chunking", "hdg_set_chunk_buffers",
           "hdg_set_factor_store", "hdg_factor_store_macros", "hdg_set_progress",
           "hdg_autotune", "hdg_class_count", "hdg_get_tuning", "hdg_set_tuning",
           "hdg_condense_first_layer", "hdg_flow_diagnostics", "hdg_flow_diagnostics_noalloc",
           "hdg_nested_dims", "hdg_condense_nested", "hdg_nested_solve"]

_lib = None


def load_library(path=LIB_PATH):
    """Load libhdg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2402_11361_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, dp, sz, i = ctypes.c_void_p, ctypes.c_double, ctypes.c_size_t, ctypes.c_int
    lib.hdg_setup_mesh.argtypes = [ctypes.POINTER(_MeshDesc), ctypes.POINTER(_Phys), vp, ctypes.POINTER(vp)]
    lib.hdg_query_sizes.argtypes = [vp, ctypes.POINTER(_Sizes)]
    lib.hdg_macro_offsets.argtypes = [vp, vp, vp]
    lib.hdg_face_offsets.argtypes = [vp, vp]
    lib.hdg_node_coords.argtypes = [vp, vp, vp]
    lib.hdg_bind_workspace.argtypes = [vp, vp, sz]
    lib.hdg_set_chunking.argtypes = [vp, i]
    lib.hdg_set_chunk_buffers.argtypes = [vp, i]
    lib.hdg_set_factor_store.argtypes = [vp, i, i]
    lib.hdg_factor_store_macros.argtypes = [vp, ctypes.POINTER(i)]
    lib.hdg_set_progress.argtypes = [vp, i]
    ip = ctypes.POINTER(ctypes.c_int)
    lib.hdg_autotune.argtypes = [vp, i, ctypes.c_char_p, ip]
    lib.hdg_class_count.argtypes = [vp, ip]
    lib.hdg_get_tuning.argtypes = [vp, i, i, ip, ip, ip]
    lib.hdg_set_tuning.argtypes = [vp, i, i, i, i, i]
    lib.hdg_linearize_stage.argtypes = [vp, vp, vp, vp, vp, dp, dp, dp, vp]
    lib.hdg_condense.argtypes = [vp, i, vp]
    lib.hdg_condense_first_layer.argtypes = [vp, vp]
    lib.hdg_nested_dims.argtypes = [vp, i, ip, ip, ip]
    lib.hdg_condense_nested.argtypes = [vp, i, vp, vp]
    lib.hdg_nested_solve.argtypes = [vp, i, vp, ctypes.POINTER(KrylovOpts), ctypes.POINTER(KrylovStats)]
    lib.hdg_flow_diagnostics.argtypes = [vp, vp, vp, vp]
    lib.hdg_flow_diagnostics_noalloc.argtypes = [vp, vp, vp, vp]
    lib.hdg_apply_global.argtypes = [vp, vp, vp]
    lib.hdg_fgmres_solve.argtypes = [vp, vp, vp, ctypes.POINTER(KrylovOpts), ctypes.POINTER(KrylovStats)]
    lib.hdg_local_backsolve.argtypes = [vp, vp, vp, vp]
    lib.hdg_axpy.argtypes = [vp, sz, dp, vp, vp]
    lib.hdg_destroy.argtypes = [vp]
    lib.hdg_status_string.argtypes = [i]
    lib.hdg_status_string.restype = ctypes.c_char_p
    lib.hdg_last_error.argtypes = [vp]
    lib.hdg_last_error.restype = ctypes.c_char_p
    lib.hdg_get_condensed.argtypes = [vp, sz, vp, vp]
    lib.hdg_get_formed.argtypes = [vp, sz, vp]
    lib.hdg_get_residuals.argtypes = [vp, vp, vp, vp]
    fl = ctypes.c_float
    mp = ctypes.POINTER(Mlp)
    lib.hdg_precond_apply.argtypes = [vp, vp, vp, i, i, i]
    lib.hdg_coarse_size.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.hdg_coarse_restrict.argtypes = [vp, vp, vp]
    lib.hdg_coarse_neighbours.argtypes = [vp, vp, vp]
    lib.hdg_coarse_prolong.argtypes = [vp, vp, dp, vp]
    lib.hdg_mlp_param_count.argtypes = [i, i, i]
    lib.hdg_mlp_work_floats.argtypes = [i, i, i, i]
    lib.hdg_mlp_forward.argtypes = [vp, mp, vp, vp, i, vp]
    lib.hdg_mlp_loss_grad.argtypes = [vp, mp, vp, vp, vp, i, vp]
    lib.hdg_mlp_adam.argtypes = [vp, mp, fl, fl, fl, fl, i]
    lib.hdg_learned_bind.argtypes = [vp, mp]
    for name in EXPORTS:
        if name not in ("hdg_status_string", "hdg_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    lib.hdg_mlp_param_count.restype = ctypes.c_size_t
    lib.hdg_mlp_work_floats.restype = ctypes.c_size_t
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """One mesh + physics set-up (hdg_setup_mesh) with its bound workspace."""

    def __init__(self, dim, n_elem, lo, hi, periodic, seg_len, p, gamma=1.4, Pr=0.71, Re=100.0, Mach=0.1,
                 supg=False, bc_state=None, stream=None):
        import torch
        self.lib = load_library()
        self.torch = torch
        md = _MeshDesc()
        md.dim = dim
        md.p = p
        self._segs = []
        for k in range(3):
            if k < dim:
                seg = np.ascontiguousarray(seg_len[k], dtype=np.int32)
                self._segs.append(seg)
                md.n_elem[k] = int(n_elem[k])
                md.lo[k] = float(lo[k])
                md.hi[k] = float(hi[k])
                md.periodic[k] = int(bool(periodic[k]))
                md.n_seg[k] = seg.size
                md.seg_len[k] = seg.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
            else:
                md.n_elem[k] = 1
                md.n_seg[k] = 1
        ph = _Phys()
        ph.gamma, ph.Pr, ph.Re, ph.Mach, ph.supg = gamma, Pr, Re, Mach, int(supg)
        self._bc = None
        if bc_state is not None:
            self._bc = np.ascontiguousarray(bc_state, dtype=np.float64)
            ph.bc_state_host = self._bc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(self.lib.hdg_setup_mesh(ctypes.byref(md), ctypes.byref(ph), ctypes.c_void_p(stream),
                                            ctypes.byref(h)), ctx=None)
        self.h = h
        s = _Sizes()
        self._check(self.lib.hdg_query_sizes(self.h, ctypes.byref(s)))
        self.n_macros, self.n_glob = s.n_macros, s.n_glob
        self.n_u_tot, self.n_q_tot = s.n_u_tot, s.n_q_tot
        self.n_u_macro, self.n_b_macro = s.n_u_macro, s.n_b_macro
        self.workspace_bytes = s.workspace_bytes
        self.chunk_macros = 0
        self.chunk_buffers = 1
        self.dim = dim
        self.ws = None
        # per-macro offsets in u (q: dim * u_off) and in the local trace vectors
        self.u_off = np.zeros(self.n_macros + 1, dtype=np.int64)
        self.b_off = np.zeros(self.n_macros + 1, dtype=np.int64)
        self._check(self.lib.hdg_macro_offsets(self.h, _np_ptr(self.u_off), _np_ptr(self.b_off)))
        self.n_faces = s.n_faces
        self.face_off = np.zeros(self.n_faces + 1, dtype=np.int64)
        self._check(self.lib.hdg_face_offsets(self.h, _np_ptr(self.face_off)))

    def _check(self, code, ctx="self"):
        if code != 0:
            msg = self.lib.hdg_last_error(self.h).decode() if ctx == "self" else ""
            raise HdgError(code, msg or self.lib.hdg_status_string(code).decode())

    @classmethod
    def from_mesh_spec(cls, spec, **kw):
        return cls(spec["dim"], spec["n_elem"], spec["lo"], spec["hi"], spec["periodic"], spec["seg_len"], spec["p"], **kw)

    def set_chunking(self, macros_per_chunk):
        """Condense in ranges of macros_per_chunk macros (0: all at once; the
        first range takes the remainder).  Re-plans the workspace;
        bind_workspace() must follow."""
        self._check(self.lib.hdg_set_chunking(self.h, int(macros_per_chunk)))
        self.ws = None
        s = _Sizes()
        self._check(self.lib.hdg_query_sizes(self.h, ctypes.byref(s)))
        self.workspace_bytes = s.workspace_bytes
        self.chunk_macros = int(macros_per_chunk)

    def set_chunk_buffers(self, n_buffers):
        """Chunk slots of W (1 or 2; with 2 the next chunk is formed beside
        the elimination of this one).  Re-plans the workspace like
        set_chunking; bind_workspace() must follow."""
        self._check(self.lib.hdg_set_chunk_buffers(self.h, int(n_buffers)))
        self.ws = None
        s = _Sizes()
        self._check(self.lib.hdg_query_sizes(self.h, ctypes.byref(s)))
        self.workspace_bytes = s.workspace_bytes
        self.chunk_buffers = int(n_buffers)

    def set_factor_store(self, n_macros, prec=None):
        """Keep the S factors of up to n_macros macros (whole leading chunks)
        from the condensation for the recovery, in prec (HDG_FP32 default or
        HDG_FP64).  Re-plans the workspace; bind_workspace() must follow.
        Returns the number of macros the plan keeps."""
        prec = HDG_FP32 if prec is None else prec
        self._check(self.lib.hdg_set_factor_store(self.h, int(n_macros), int(prec)))
        self.ws = None
        s = _Sizes()
        self._check(self.lib.hdg_query_sizes(self.h, ctypes.byref(s)))
        self.workspace_bytes = s.workspace_bytes
        n = ctypes.c_int(0)
        self._check(self.lib.hdg_factor_store_macros(self.h, ctypes.byref(n)))
        self.store_macros = n.value
        return n.value

    def set_progress(self, on=True):
        """Progress lines on stderr per finished chunk of the condensation and
        the recovery (waits for the stream after each chunk)."""
        self._check(self.lib.hdg_set_progress(self.h, 1 if on else 0))

    def fit_factor_store(self, budget_bytes, prec=None):
        """Largest factor store (in macros) whose workspace fits in
        budget_bytes under the current chunking; returns the macros kept."""
        lo, hi, best = 0, self.n_macros, 0
        while lo <= hi:
            mid = (lo + hi) // 2
            self.set_factor_store(mid, prec)
            if self.workspace_bytes <= budget_bytes:
                best, lo = mid, mid + 1
            else:
                hi = mid - 1
        return self.set_factor_store(best, prec)

    def fit_chunking(self, budget_bytes):
        """Largest macros per chunk (0 = no chunking) whose workspace fits in
        budget_bytes; returns it after applying it."""
        if self.workspace_bytes <= budget_bytes and self.chunk_macros == 0:
            return 0
        lo, hi = 1, self.n_macros
        self.set_chunking(0)
        if self.workspace_bytes <= budget_bytes:
            return 0
        best = None
        while lo <= hi:
            mid = (lo + hi) // 2
            self.set_chunking(mid)
            if self.workspace_bytes <= budget_bytes:
                best, lo = mid, mid + 1
            else:
                hi = mid - 1
        if best is None:
            raise HdgError(2, f"workspace does not fit in {budget_bytes} bytes even with one macro per chunk")
        self.set_chunking(best)
        return best

    def autotune(self, prec=HDG_FP64, cache_path=None):
        """Pick the elimination launch shapes per macro class (needs a
        linearisation; condense afterwards).  Returns the number of classes
        timed (the others came from cache_path)."""
        n = ctypes.c_int(0)
        cp = None if cache_path is None else os.fsencode(cache_path)
        self._check(self.lib.hdg_autotune(self.h, prec, cp, ctypes.byref(n)))
        return n.value

    def class_count(self):
        n = ctypes.c_int(0)
        self._check(self.lib.hdg_class_count(self.h, ctypes.byref(n)))
        return n.value

    def tuning(self, macro_class, prec=HDG_FP64):
        """(tiles per workgroup, panel kind, look-ahead stream) of a class."""
        tpw, panel, look = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        self._check(self.lib.hdg_get_tuning(self.h, macro_class, prec, ctypes.byref(tpw), ctypes.byref(panel),
                                            ctypes.byref(look)))
        return tpw.value, panel.value, look.value

    def set_tuning(self, macro_class, prec, tpw, panel=0, lookahead=0):
        self._check(self.lib.hdg_set_tuning(self.h, macro_class, prec, tpw, panel, lookahead))

    def bind_workspace(self, ws=None):
        """Allocate (torch) and bind the device workspace."""
        t = self.torch
        if ws is None:
            ws = t.empty(self.workspace_bytes + 256, dtype=t.uint8, device="cuda")
        base = ws.data_ptr()
        off = (-base) % 256
        self.ws = ws
        self._check(self.lib.hdg_bind_workspace(self.h, ctypes.c_void_p(base + off), ctypes.c_size_t(ws.numel() - off)))
        return ws

    def node_coords(self):
        d = self.dim
        mx = np.zeros(self.n_u_tot // (d + 2) * d)
        fx = np.zeros(self.n_glob // (d + 2) * d)
        self._check(self.lib.hdg_node_coords(self.h, _np_ptr(mx), _np_ptr(fx)))
        return mx.reshape(-1, d), fx.reshape(-1, d)

    def node_coords_split(self):
        """Node coordinates as lists: one [N_i, d] array per macro and one
        [n_nodes_f, d] array per face."""
        mx, fx = self.node_coords()
        ns = self.dim + 2
        mo = self.u_off // ns
        fo = self.face_off // ns
        return ([mx[mo[i]:mo[i + 1]] for i in range(self.n_macros)],
                [fx[fo[f]:fo[f + 1]] for f in range(self.n_faces)])

    def linearize_stage(self, q, u, uhat, w=None, dt=math.inf, d_ii=1.0, dtau=math.inf, norms=True):
        out = np.zeros(3) if norms else None
        self._check(self.lib.hdg_linearize_stage(self.h, _ptr(q), _ptr(u), _ptr(uhat), _ptr(w), dt, d_ii, dtau,
                                                 _np_ptr(out) if norms else None))
        return out

    def condense(self, bhat, prec=HDG_FP64):
        self._check(self.lib.hdg_condense(self.h, prec, _ptr(bhat)))

    def condense_first_layer(self, bhat):
        """Standard (first-layer) condensation of (q, u) together (chunked,
        one macro shape); same A-hat and b-hat as condense()."""
        self._check(self.lib.hdg_condense_first_layer(self.h, _ptr(bhat)))


    def nested_dims(self, block_m):
        """(blocks, internal-face and boundary-face trace unknowns per block) of
        the nested condensation with blocks of block_m elements per axis."""
        nb, ni, nbd = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        self._check(self.lib.hdg_nested_dims(self.h, block_m, ctypes.byref(nb), ctypes.byref(ni), ctypes.byref(nbd)))
        return nb.value, ni.value, nbd.value

    def condense_nested(self, block_m, ahat, bhat):
        """A-hat^G (n_blocks x n_B x n_B) and b-hat^G (n_blocks x n_B) into
        the given float64 device tensors."""
        nb, _, nbd = self.nested_dims(block_m)
        if ahat.numel() != nb * nbd * nbd or bhat.numel() != nb * nbd:
            raise ValueError("ahat / bhat sizes do not match hdg_nested_dims")
        self._check(self.lib.hdg_condense_nested(self.h, block_m, _ptr(ahat), _ptr(bhat)))

    def nested_solve(self, block_m, x_full, rtol=1e-8, atol=0.0, restart=30, max_outer=300, inner_its=5,
                     allow_noconv=False):
        """FGMRES on the block skeleton of the last condense_nested, then the
        internal-face traces: the whole element-trace increment in x_full."""
        if x_full.numel() != self.n_glob:
            raise ValueError("x_full must hold n_glob values")
        o = KrylovOpts(rtol, atol, restart, max_outer, inner_its, HDG_FP64, 0, 0, None, 0, 0)
        st = KrylovStats()
        code = self.lib.hdg_nested_solve(self.h, block_m, _ptr(x_full), ctypes.byref(o), ctypes.byref(st))
        if not (allow_noconv and code == 5):
            self._check(code)
        return dict(outer_its=st.outer_its, inner_its=st.inner_its_total, res0=st.res0, res=st.res_final,
                    ms=st.ms, converged=(code == 0))
    def flow_diagnostics(self, q, u):
        """(E_k, eps, |Omega|): volume-averaged kinetic energy and the
        dissipation rate of eq. C5321 of the state (q, u), library units."""
        out = np.zeros(3)
        self._check(self.lib.hdg_flow_diagnostics(self.h, _ptr(q), _ptr(u), _np_ptr(out)))
        return float(out[0]), float(out[1]), float(out[2])

    def flow_diagnostics_noalloc(self, q, u):
        """flow_diagnostics through the entry point that allocates nothing
        (static device scratch; no workspace needed)."""
        out = np.zeros(3)
        self._check(self.lib.hdg_flow_diagnostics_noalloc(self.h, _ptr(q), _ptr(u), _np_ptr(out)))
        return float(out[0]), float(out[1]), float(out[2])

    def apply_global(self, x, y):
        self._check(self.lib.hdg_apply_global(self.h, _ptr(x), _ptr(y)))

    def fgmres_solve(self, b, x, rtol=1e-8, atol=0.0, restart=30, max_outer=300, inner_its=5,
                     inner_prec=HDG_FP64, allow_noconv=False, use_learned=False, harvest=None, graph_steps=0,
                     no_fallback=False):
        """harvest: optional device tensor [k, n_glob] receiving the vectors the
        preconditioner is applied to (first k).  graph_steps > 0: device-resident
        Arnoldi steps replayed from HIP graphs of that many steps.  no_fallback:
        keep the learned stage for the whole solve."""
        hv = _ptr(harvest) if harvest is not None else None
        hk = int(harvest.shape[0]) if harvest is not None else 0
        o = KrylovOpts(rtol, atol, restart, max_outer, inner_its, inner_prec, int(bool(use_learned)),
                       int(bool(no_fallback)), hv, hk, int(graph_steps))
        st = KrylovStats()
        code = self.lib.hdg_fgmres_solve(self.h, _ptr(b), _ptr(x), ctypes.byref(o), ctypes.byref(st))
        if not (allow_noconv and code == 5):
            self._check(code)
        return dict(outer_its=st.outer_its, inner_its=st.inner_its_total, res0=st.res0, res=st.res_final,
                    ms=st.ms, converged=(code == 0), fallbacks=st.fallbacks, harvested=st.harvested)

    def precond_apply(self, v, z, inner_its=5, inner_prec=HDG_FP64, use_learned=False):
        self._check(self.lib.hdg_precond_apply(self.h, _ptr(v), _ptr(z), inner_its, inner_prec, int(bool(use_learned))))

    def coarse_size(self):
        n = ctypes.c_int()
        self._check(self.lib.hdg_coarse_size(self.h, ctypes.byref(n)))
        return n.value

    def coarse_restrict(self, v, X):
        self._check(self.lib.hdg_coarse_restrict(self.h, _ptr(v), _ptr(X)))

    def coarse_neighbours(self, X, Xe):
        """Xe = [own | face neighbours'] coarse coefficients per macro."""
        self._check(self.lib.hdg_coarse_neighbours(self.h, _ptr(X), _ptr(Xe)))

    def coarse_prolong(self, Y, alpha, z):
        self._check(self.lib.hdg_coarse_prolong(self.h, _ptr(Y), float(alpha), _ptr(z)))

    def mlp_forward(self, net, X, idx, batch, Y):
        self._check(self.lib.hdg_mlp_forward(self.h, ctypes.byref(net), _ptr(X), _ptr(idx), int(batch), _ptr(Y)))

    def mlp_loss_grad(self, net, X, T, idx, batch, loss):
        self._check(self.lib.hdg_mlp_loss_grad(self.h, ctypes.byref(net), _ptr(X), _ptr(T), _ptr(idx), int(batch),
                                               _ptr(loss)))

    def mlp_adam(self, net, lr, beta1, beta2, eps, step):
        self._check(self.lib.hdg_mlp_adam(self.h, ctypes.byref(net), lr, beta1, beta2, eps, int(step)))

    def learned_bind(self, net):
        self._check(self.lib.hdg_learned_bind(self.h, ctypes.byref(net) if net is not None else None))

    def local_backsolve(self, duhat, dq, du):
        self._check(self.lib.hdg_local_backsolve(self.h, _ptr(duhat), _ptr(dq), _ptr(du)))

    def axpy(self, a, x, y):
        self._check(self.lib.hdg_axpy(self.h, ctypes.c_size_t(x.numel()), float(a), _ptr(x), _ptr(y)))

    def get_condensed(self, macro):
        nb = int(self.b_off[macro + 1] - self.b_off[macro])
        A = np.zeros((nb, nb))
        b = np.zeros(nb)
        self._check(self.lib.hdg_get_condensed(self.h, ctypes.c_size_t(macro), _np_ptr(A), _np_ptr(b)))
        return A, b

    def get_formed(self, macro):
        nr = int(self.u_off[macro + 1] - self.u_off[macro] + self.b_off[macro + 1] - self.b_off[macro])
        W = np.zeros((nr, nr + 1))
        self._check(self.lib.hdg_get_formed(self.h, ctypes.c_size_t(macro), _np_ptr(W)))
        return W

    def get_residuals(self):
        t = self.torch
        rq = t.empty(self.n_q_tot, dtype=t.float64, device="cuda")
        ru = t.empty(self.n_u_tot, dtype=t.float64, device="cuda")
        rb = t.empty(self.n_glob, dtype=t.float64, device="cuda")
        self._check(self.lib.hdg_get_residuals(self.h, _ptr(rq), _ptr(ru), _ptr(rb)))
        return rq, ru, rb

    def close(self):
        if getattr(self, "h", None):
            self.lib.hdg_destroy(self.h)
            self.h = None
        self.ws = None  # the workspace goes back to torch's allocator

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mesh_spec_box(dim, n_elem, m, p, lo, hi, periodic):
    n_elem = [n_elem] * dim if np.isscalar(n_elem) else list(n_elem)
    m = [m] * dim if np.isscalar(m) else list(m)
    lo = [lo] * dim if np.isscalar(lo) else list(lo)
    hi = [hi] * dim if np.isscalar(hi) else list(hi)
    per = [periodic] * dim if np.isscalar(periodic) else list(periodic)
    seg = [[m[k]] * (n_elem[k] // m[k]) for k in range(dim)]
    return dict(dim=dim, n_elem=n_elem, lo=lo, hi=hi, periodic=per, seg_len=seg, p=p)

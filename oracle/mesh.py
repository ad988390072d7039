"""Box mesh grouped into box macro-elements; macro skeleton faces.
Test infrastructure (oracle).

Paper Sec. 2.2 (mesh, patches Omega_i, interfaces Gamma_i) and Sec. 2.2 spaces:
u and q are C0 within each macro-element, the trace u-hat lives on the macro
skeleton.  Reading: macro-elements are axis-aligned boxes of m_x x m_y (x m_z)
tensor-product elements of degree p (the paper uses simplices); the trace on a
macro face is C0 Q_p on that face's sub-faces and each macro face carries its
own trace nodes (trace space per face e of the skeleton).  With a degree per
macro, a face between degrees p+ and p- carries C0 Q_max(p+, p-).

Numbering (shared convention with the HIP library, fixed here by hand):
  * macro (s_0, s_1[, s_2]) -> s_0 + n_seg0 * (s_1 + n_seg1 * s_2)
  * macro node (i_0, i_1[, i_2]) -> i_0 + n_0 * (i_1 + n_1 * i_2), n_k = m_k p + 1
    (p the macro's degree)
  * u layout [macro][comp][node]; q layout [macro][dir][comp][node]
  * faces: all faces normal to axis 0, then axis 1, then axis 2; within axis k
    the face grid has nb_k positions along k (n_seg_k if periodic else
    n_seg_k + 1) and n_seg_j along the other axes, enumerated lexicographically
    with axis 0 fastest
  * face node (t_0, t_1) over the tangential axes in increasing order,
    t_0 fastest; global trace layout [face][comp][facenode]
  * a macro's 2d local faces ordered (k=0,s=0), (k=0,s=1), (k=1,s=0), ...
    where s=0 is the low side along k.
"""
import numpy as np
from .basis import gll_nodes


class Mesh:
    def __init__(self, dim, n_elem, lo, hi, periodic, seg_len, p, macro_p=None):
        """macro_p: optional polynomial degree per macro (mixed degrees); the
        trace on a face between macros of degrees p+ and p- then has degree
        max(p+, p-), so that it contains the traces of both sides."""
        self.dim = d = int(dim)
        self.p = int(p)
        self.n_elem = [int(n_elem[k]) for k in range(d)]
        self.lo = [float(lo[k]) for k in range(d)]
        self.hi = [float(hi[k]) for k in range(d)]
        self.periodic = [bool(periodic[k]) for k in range(d)]
        self.seg_len = [np.asarray(seg_len[k], dtype=int) for k in range(d)]
        for k in range(d):
            if self.seg_len[k].sum() != self.n_elem[k]:
                raise ValueError("segments must cover the mesh")
        self.h = [(self.hi[k] - self.lo[k]) / self.n_elem[k] for k in range(d)]
        self.n_seg = [len(self.seg_len[k]) for k in range(d)]
        self.seg_start = [np.concatenate([[0], np.cumsum(self.seg_len[k])[:-1]]) for k in range(d)]
        self.ns = d + 2
        self.n_macros = int(np.prod(self.n_seg))
        self.macro_p = (np.full(self.n_macros, self.p, dtype=int) if macro_p is None
                        else np.asarray(macro_p, dtype=int).reshape(-1))
        if self.macro_p.size != self.n_macros or self.macro_p.min() < 1:
            raise ValueError("macro_p needs one degree >= 1 per macro")
        self.mixed = bool((self.macro_p != self.p).any())
        self._build_faces()

    # ---- macros -------------------------------------------------------
    def macro_seg(self, i):
        s = []
        for k in range(self.dim):
            s.append(i % self.n_seg[k])
            i //= self.n_seg[k]
        return s

    def macro_index(self, s):
        i = 0
        for k in reversed(range(self.dim)):
            i = i * self.n_seg[k] + s[k]
        return i

    def macro_m(self, i):
        s = self.macro_seg(i)
        return [int(self.seg_len[k][s[k]]) for k in range(self.dim)]

    def macro_deg(self, i):
        return int(self.macro_p[i])

    def face_deg(self, f):
        """Trace degree of face f: the larger degree of the macros beside it."""
        return int(self.faces[f]["deg"])

    def macro_face_degs(self, i):
        """Trace degrees of macro i's 2d local faces in local order."""
        return [self.face_deg(self.macro_faces[i, lf]) for lf in range(2 * self.dim)]

    def macro_nodes_1d(self, i):
        """Per axis: node counts n_k = m_k p_i + 1."""
        return [m * self.macro_deg(i) + 1 for m in self.macro_m(i)]

    def macro_n_nodes(self, i):
        return int(np.prod(self.macro_nodes_1d(i)))

    def macro_node_coords(self, i):
        """[N, d] physical coordinates of the C0 macro nodes (GLL in each element)."""
        s = self.macro_seg(i)
        pi = self.macro_deg(i)
        g = gll_nodes(pi)
        axes = []
        for k in range(self.dim):
            m = self.seg_len[k][s[k]]
            x0 = self.lo[k] + self.seg_start[k][s[k]] * self.h[k]
            pts = [x0 + self.h[k] * (e + (g[j] + 1.0) / 2.0)
                   for e in range(m) for j in range(pi + 1) if not (e > 0 and j == 0)]
            axes.append(np.array(pts))
        grids = np.meshgrid(*axes, indexing="ij")
        # lexicographic with axis 0 fastest -> transpose of C order
        return np.stack([gk.transpose().reshape(-1) for gk in grids], axis=1)

    # ---- faces --------------------------------------------------------
    def _build_faces(self):
        d = self.dim
        faces = []  # dicts
        self.macro_faces = np.full((self.n_macros, 2 * d), -1, dtype=int)
        for k in range(d):
            nb = self.n_seg[k] if self.periodic[k] else self.n_seg[k] + 1
            dims = [nb if j == k else self.n_seg[j] for j in range(d)]
            for flat in range(int(np.prod(dims))):
                c = []
                t = flat
                for j in range(d):
                    c.append(t % dims[j])
                    t //= dims[j]
                b = c[k]
                minus = plus = -1
                if self.periodic[k]:
                    sm = list(c); sm[k] = (b - 1) % self.n_seg[k]
                    sp = list(c); sp[k] = b
                    minus = self.macro_index(sm)
                    plus = self.macro_index(sp)
                else:
                    if b > 0:
                        sm = list(c); sm[k] = b - 1
                        minus = self.macro_index(sm)
                    if b < self.n_seg[k]:
                        sp = list(c); sp[k] = b
                        plus = self.macro_index(sp)
                tang = [j for j in range(d) if j != k]
                deg = max(int(self.macro_p[i]) for i in (minus, plus) if i >= 0)
                tn = [int(self.seg_len[j][c[j]]) * deg + 1 for j in tang]
                fid = len(faces)
                faces.append(dict(axis=k, minus=minus, plus=plus, tang=tang, deg=deg,
                                  tn=tn, n_nodes=int(np.prod(tn)), grid=c))
                if minus >= 0:
                    self.macro_faces[minus, 2 * k + 1] = fid
                if plus >= 0:
                    self.macro_faces[plus, 2 * k + 0] = fid
        self.faces = faces
        self.n_faces = len(faces)
        self.face_ndof = np.array([self.ns * f["n_nodes"] for f in faces], dtype=int)
        self.face_offset = np.concatenate([[0], np.cumsum(self.face_ndof)[:-1]]).astype(int)
        self.n_glob = int(self.face_ndof.sum())

    def face_is_boundary(self, f):
        fc = self.faces[f]
        return fc["minus"] < 0 or fc["plus"] < 0

    def macro_face_nodes(self, i, lf):
        """Macro node ids lying on local face lf = 2k+s, in face-node order."""
        d = self.dim
        k, s = divmod(lf, 2)
        n = self.macro_nodes_1d(i)
        tang = [j for j in range(d) if j != k]
        fixed = 0 if s == 0 else n[k] - 1
        ids = []
        if d == 2:
            for t0 in range(n[tang[0]]):
                idx = [0, 0]; idx[k] = fixed; idx[tang[0]] = t0
                ids.append(idx[0] + n[0] * idx[1])
        else:
            for t1 in range(n[tang[1]]):
                for t0 in range(n[tang[0]]):
                    idx = [0, 0, 0]; idx[k] = fixed; idx[tang[0]] = t0; idx[tang[1]] = t1
                    ids.append(idx[0] + n[0] * (idx[1] + n[1] * idx[2]))
        return np.array(ids, dtype=int)

    def face_node_coords(self, f):
        """[n_nodes, d] coordinates of the trace nodes of face f (taken from the
        plus-side macro if present and of the face's degree, else the minus
        side: a side of the face's degree has its face nodes at the trace
        nodes)."""
        fc = self.faces[f]
        if fc["plus"] >= 0 and self.macro_deg(fc["plus"]) == fc["deg"]:
            i, lf = fc["plus"], 2 * fc["axis"]
        else:
            i, lf = fc["minus"], 2 * fc["axis"] + 1
        X = self.macro_node_coords(i)
        return X[self.macro_face_nodes(i, lf)]

    def macro_trace_index(self, i):
        """Global trace-dof indices of macro i's local boundary vector
        (its 2d faces in local order, each [comp][facenode])."""
        idx = []
        for lf in range(2 * self.dim):
            f = self.macro_faces[i, lf]
            idx.append(self.face_offset[f] + np.arange(self.face_ndof[f]))
        return np.concatenate(idx)


def box_mesh(dim, n_elem, m, p, lo=None, hi=None, periodic=False, macro_p=None):
    """Uniform segmentation: every macro has m elements per axis (macro_p:
    optional degree per macro)."""
    n_elem = [n_elem] * dim if np.isscalar(n_elem) else list(n_elem)
    m = [m] * dim if np.isscalar(m) else list(m)
    lo = [0.0] * dim if lo is None else (list(lo) if not np.isscalar(lo) else [lo] * dim)
    hi = [1.0] * dim if hi is None else (list(hi) if not np.isscalar(hi) else [hi] * dim)
    per = [periodic] * dim if np.isscalar(periodic) else list(periodic)
    seg = []
    for k in range(dim):
        if n_elem[k] % m[k]:
            raise ValueError("n_elem must be a multiple of m")
        seg.append([m[k]] * (n_elem[k] // m[k]))
    return Mesh(dim, n_elem, lo, hi, per, seg, p, macro_p)

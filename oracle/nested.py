"""Nested hybridisation inside a macro: a third static-condensation layer.
Test infrastructure (oracle).

An alternative local structure to the paper's C0 macro (Sec. 2.2 builds each
patch T_i from elements and hybridises only on the patch boundaries).  Here
every element is hybridised on its own: u and q are discontinuous between
elements and every element face carries a trace.  That is the macro-element
method with one element per macro (m = 1), whose condensed blocks are the
element blocks A-hat^{T_e}, b-hat^{T_e} of eq. (C44).  The elements are then
grouped into blocks of M elements per axis.  Per block G, the element blocks
are assembled over the faces of G's elements, and the traces of the faces
inside G are eliminated (static condensation once more, as in eq. ASC2):

    A_G = [[A_II, A_IB], [A_BI, A_BB]],  b_G = [b_I; b_B]
    A-hat^G = A_BB - A_BI A_II^{-1} A_IB,  b-hat^G = b_B - A_BI A_II^{-1} b_I

which leaves a global system on the block skeleton only (the faces between
blocks and on the domain boundary), assembled like eq. (C44).  The traces of
the internal faces follow from the skeleton traces block by block,
x_I = A_II^{-1} (b_I - A_IB x_B), and the element unknowns from all traces by
the local recovery of eq. (Csc4).

Block numbering: block (g_0, g_1[, g_2]) -> g_0 + n_0 (g_1 + n_1 g_2), element
(macro) s -> block (s_k // M).  Block-local trace order: the internal faces of
the block in increasing global face id, then its boundary faces in increasing
global face id; each face's dofs in their global order.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def internal_trace_dofs(dim, M, p):
    """Trace dofs on the faces inside one block of M^dim elements of degree p:
    dim (M - 1) M^(dim - 1) internal faces, (p + 1)^(dim - 1) nodes and
    dim + 2 components each."""
    return dim * (M - 1) * M ** (dim - 1) * (p + 1) ** (dim - 1) * (dim + 2)


class Blocks:
    """Grouping of the elements of a one-element-per-macro box mesh into
    blocks of M elements per axis."""

    def __init__(self, mesh, M):
        d = mesh.dim
        for k in range(d):
            if any(int(s) != 1 for s in mesh.seg_len[k]):
                raise ValueError("nested blocks need one element per macro")
            if mesh.n_seg[k] % M:
                raise ValueError("the element count per axis must be a multiple of M")
        self.mesh, self.M = mesh, M
        self.n_blk_axis = [mesh.n_seg[k] // M for k in range(d)]
        self.n_blocks = int(np.prod(self.n_blk_axis))
        self.block_of = np.array([self._block(mesh.macro_seg(i)) for i in range(mesh.n_macros)])
        self.elements = [np.flatnonzero(self.block_of == g) for g in range(self.n_blocks)]
        # faces of each block: internal (both sides in the block) and boundary
        side_blocks = {}
        for f, fc in enumerate(mesh.faces):
            side_blocks[f] = [self.block_of[m] for m in (fc["minus"], fc["plus"]) if m >= 0]
        self.internal, self.boundary = [], []
        for g in range(self.n_blocks):
            fs = sorted({int(mesh.macro_faces[e, lf]) for e in self.elements[g] for lf in range(2 * d)})
            self.internal.append([f for f in fs if len(side_blocks[f]) == 2 and all(b == g for b in side_blocks[f])])
            self.boundary.append([f for f in fs if f not in set(self.internal[-1])])
        # skeleton: faces that are not internal to any block, in global order
        inner = set(f for fl in self.internal for f in fl)
        self.skeleton = [f for f in range(mesh.n_faces) if f not in inner]
        off = np.zeros(mesh.n_faces, dtype=int)
        pos = 0
        for f in self.skeleton:
            off[f] = pos
            pos += mesh.face_ndof[f]
        self.skel_off, self.n_skel = off, pos

    def _block(self, s):
        g = 0
        for k in reversed(range(self.mesh.dim)):
            g = g * self.n_blk_axis[k] + s[k] // self.M
        return g

    def face_dofs(self, faces):
        m = self.mesh
        return np.concatenate([m.face_offset[f] + np.arange(m.face_ndof[f]) for f in faces]) if faces else \
            np.zeros(0, dtype=int)

    def skel_dofs(self, faces):
        m = self.mesh
        return np.concatenate([self.skel_off[f] + np.arange(m.face_ndof[f]) for f in faces])

    def local_system(self, cond, g):
        """A_G and b_G of block g assembled from the element blocks (global
        trace dofs of the block: internal faces, then boundary faces)."""
        m = self.mesh
        gI, gB = self.face_dofs(self.internal[g]), self.face_dofs(self.boundary[g])
        glob = np.concatenate([gI, gB])
        where = {int(x): i for i, x in enumerate(glob)}
        n = glob.size
        A = np.zeros((n, n))
        b = np.zeros(n)
        for e in self.elements[g]:
            loc = np.array([where[int(x)] for x in m.macro_trace_index(e)])
            A[np.ix_(loc, loc)] += cond[e]["Ahat"]
            b[loc] += cond[e]["bhat"]
        return A, b, gI.size


def condense(blocks, cond):
    """Per block: A-hat^G and b-hat^G on its boundary faces, with the LU of
    A_II and the coupling blocks kept for the recovery of the internal traces."""
    out = []
    for g in range(blocks.n_blocks):
        A, b, nI = blocks.local_system(cond, g)
        AII, AIB, ABI, ABB = A[:nI, :nI], A[:nI, nI:], A[nI:, :nI], A[nI:, nI:]
        if nI:
            lu = sla.lu_factor(AII)
            Ahat = ABB - ABI @ sla.lu_solve(lu, AIB)
            bhat = b[nI:] - ABI @ sla.lu_solve(lu, b[:nI])
        else:
            lu, Ahat, bhat = None, ABB.copy(), b.copy()
        out.append(dict(Ahat=Ahat, bhat=bhat, lu=lu, AIB=AIB, bI=b[:nI]))
    return out


def assemble(blocks, ncond):
    """The skeleton system: sum over blocks of their A-hat^G, b-hat^G."""
    rows, cols, vals = [], [], []
    b = np.zeros(blocks.n_skel)
    for g, C in enumerate(ncond):
        idx = blocks.skel_dofs(blocks.boundary[g])
        rows.append(np.repeat(idx, idx.size))
        cols.append(np.tile(idx, idx.size))
        vals.append(C["Ahat"].reshape(-1))
        np.add.at(b, idx, C["bhat"])
    n = blocks.n_skel
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return A, b


def recover_traces(blocks, ncond, x_skel):
    """All element-face traces from the skeleton traces: the skeleton values
    in place, the internal ones x_I = A_II^{-1} (b_I - A_IB x_B) per block."""
    m = blocks.mesh
    x = np.zeros(m.n_glob)
    for f in blocks.skeleton:
        x[m.face_offset[f] + np.arange(m.face_ndof[f])] = x_skel[blocks.skel_off[f] + np.arange(m.face_ndof[f])]
    for g, C in enumerate(ncond):
        if C["lu"] is None:
            continue
        xB = x_skel[blocks.skel_dofs(blocks.boundary[g])]
        x[blocks.face_dofs(blocks.internal[g])] = sla.lu_solve(C["lu"], C["bI"] - C["AIB"] @ xB)
    return x

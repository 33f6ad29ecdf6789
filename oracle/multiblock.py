"""Multi-block hexahedral meshes and their direct stiffness summation
(oracle; test infrastructure).

A multi-block mesh is a set of macro-hexahedra (blocks), each refined into
n[0] x n[1] x n[2] cells of degree p in its own local axes, glued along whole
macro-faces in any relative orientation (Section 4.2).  The oracle
identifies nodes geometrically: block b's lattice node (I, J, K) sits at the
trilinear image of (I/(n0 p), J/(n1 p), K/(n2 p)) under the block's eight
corner points, and nodes of different blocks at the same point are one node.
On a shared face both blocks' maps reduce to the same bilinear map of its
four corners, so this is the conforming identification, with no use of
orientation flags.  DSS is then the plain S = G G^T on the cell-wise vector
(every copy receives the sum of all copies of its node), for cells in block
order, canonical [cell][local node] order within a block (cell x fastest,
local node a + (p+1)(b + (p+1)c)).
"""
from __future__ import annotations

import numpy as np


class MultiBlock:
    def __init__(self, p, block_n, corners, coords):
        """block_n: [nb][3] cells per local direction; corners: [nb][8]
        vertex ids in local corner order cx + 2 cy + 4 cz; coords: [nv][3]."""
        self.p = int(p)
        self.block_n = [tuple(int(v) for v in n) for n in block_n]
        self.corners = np.asarray(corners, dtype=int)
        self.coords = np.asarray(coords, dtype=float)
        self.nb = len(self.block_n)
        self.n1 = self.p + 1
        self._ids = None

    def block_cells(self, b):
        n = self.block_n[b]
        return n[0] * n[1] * n[2]

    def ncells(self):
        return sum(self.block_cells(b) for b in range(self.nb))

    def lattice_points(self, b):
        """Physical points of block b's lattice nodes, [N0 N1 N2, 3], x fastest."""
        n = self.block_n[b]
        p = self.p
        s = [np.arange(n[d] * p + 1) / (n[d] * p) for d in range(3)]
        K, J, I = np.meshgrid(s[2], s[1], s[0], indexing="ij")
        u, v, w = I.ravel(), J.ravel(), K.ravel()
        X = np.zeros((u.size, 3))
        for c in range(8):
            cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            wgt = (u if cx else 1 - u) * (v if cy else 1 - v) * (w if cz else 1 - w)
            X += wgt[:, None] * self.coords[self.corners[b, c]][None, :]
        return X

    def cell_node_ids(self):
        """[ncells, (p+1)^3] global node id of every cell copy (block order)."""
        if self._ids is not None:
            return self._ids
        pts = [self.lattice_points(b) for b in range(self.nb)]
        allp = np.concatenate(pts)
        key = np.round(allp * 1e8).astype(np.int64)
        _, uid = np.unique(key, axis=0, return_inverse=True)
        uid = uid.ravel()
        out = []
        off = 0
        p, n1 = self.p, self.n1
        l = np.arange(n1 ** 3)
        a, bb, c = l % n1, (l // n1) % n1, l // (n1 * n1)
        for b in range(self.nb):
            n = self.block_n[b]
            N0, N1 = n[0] * p + 1, n[1] * p + 1
            e = np.arange(self.block_cells(b))
            i, j, k = e % n[0], (e // n[0]) % n[1], e // (n[0] * n[1])
            lat = (i[:, None] * p + a) + N0 * ((j[:, None] * p + bb) + N1 * (k[:, None] * p + c))
            out.append(uid[off + lat])
            off += len(pts[b])
        self._ids = np.concatenate(out)
        return self._ids

    def nglob(self):
        return int(self.cell_node_ids().max()) + 1

    def dss(self, v_cells):
        ids = self.cell_node_ids()
        s = np.bincount(ids.ravel(), weights=np.asarray(v_cells, dtype=float).ravel(), minlength=self.nglob())
        return s[ids]


def star(p, n, k=3, height=1.0, twist=False):
    """k blocks around a common macro-edge (the z axis), each a macro-hex over
    the quad (O, H_2i, H_2i+1, H_2i+2) of the planar k-star, extruded in z.
    With `twist`, every other block lists its corners with its local x and y
    axes exchanged, so the shared faces meet with different orientations."""
    R = 1.0
    pts2 = [(0.0, 0.0)]
    for t in range(2 * k):
        ang = np.pi * t / k
        r = R if t % 2 == 0 else R * 1.3
        pts2.append((r * np.cos(ang), r * np.sin(ang)))
    # vertex ids: planar point q at z level zl -> q + (2k+1) zl
    nq = len(pts2)
    coords = [(x, y, z) for z in (0.0, height) for (x, y) in pts2]
    blocks = []
    for i in range(k):
        O, A, B, C = 0, 1 + 2 * i, 1 + (2 * i + 1) % (2 * k), 1 + (2 * i + 2) % (2 * k)
        quad = [O, A, C, B] if not (twist and i % 2) else [O, C, A, B]    # local (0,0),(1,0),(0,1),(1,1)
        blocks.append([quad[c & 3] + nq * (c >> 2) for c in range(8)])
    return MultiBlock(p, [(n, n, n)] * k, blocks, coords)


def split_cube(p, n, rng=None, m=2):
    """The unit cube cut into m^3 macro-blocks of n^3 cells; with a generator,
    every block gets a random relative orientation (a random rotation or
    reflection of its local axes), so its faces meet its neighbours' in all
    the ways an unstructured generator could produce."""
    verts = {}
    coords = []

    def vid(x, y, z):
        key = (x, y, z)
        if key not in verts:
            verts[key] = len(coords)
            coords.append((x / m, y / m, z / m))
        return verts[key]

    blocks = []
    for bz in range(m):
        for by in range(m):
            for bx in range(m):
                perm = np.arange(3) if rng is None else rng.permutation(3)
                flip = np.zeros(3, bool) if rng is None else rng.integers(0, 2, 3).astype(bool)
                cs = []
                for c in range(8):
                    loc = [(c >> d) & 1 for d in range(3)]             # local corner bits
                    glob = [0, 0, 0]
                    for d in range(3):                                 # local axis d -> global axis perm[d]
                        glob[perm[d]] = 1 - loc[d] if flip[d] else loc[d]
                    cs.append(vid(bx + glob[0], by + glob[1], bz + glob[2]))
                blocks.append(cs)
    return MultiBlock(p, [(n, n, n)] * (m ** 3), blocks, coords)

"""Mesh topology for lowest-order Nedelec elements (oracle, test infrastructure).

Section 3 of the paper discretises space with lowest-order Nedelec elements;
its nodal correction (eq. (8)) needs the discrete gradient G from the nodal H1
space into the Nedelec space. Conventions (shared with the library only by
specification):

* an edge is an unordered vertex pair stored as (tail, head) with tail < head,
  and edges are numbered by lexicographic order of (tail, head);
* the edge degree of freedom is the line integral of the field from tail to
  head, so G[e, head] = +1 and G[e, tail] = -1;
* a face (a < b < c) has boundary +[a,b] + [b,c] - [a,c], giving the discrete
  curl C (faces x edges);
* a boundary face belongs to exactly one tetrahedron; boundary edges and
  vertices are those of boundary faces; Dirichlet (u x n = 0) eliminates them.
* the Neumann condition (mu^{-1} curl u x n = 0, section 3) is natural: every
  edge stays a degree of freedom. The nodal space then contains the
  constants, which G maps to zero (G 1 = 0), so G^T M G is singular. One
  gauge vertex (the lowest-numbered one) is left out of the nodal space: the
  remaining columns of G span the same range as all of them, so the nodal
  correction (eq. (8)) is unchanged while the nodal matrix becomes SPD (for a
  connected mesh).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


DIRICHLET, NEUMANN = "dirichlet", "neumann"


class Topology:
    def __init__(self, coords: np.ndarray, tets: np.ndarray, bc: str = DIRICHLET):
        if bc not in (DIRICHLET, NEUMANN):
            raise ValueError(f"unknown boundary condition {bc!r}")
        self.bc = bc
        self.coords = np.asarray(coords, dtype=np.float64)
        self.tets = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
        nv = self.coords.shape[0]
        self.n_vertices = nv
        t = self.tets
        # edges: the 6 vertex pairs of every tet, deduplicated
        pairs = np.concatenate([t[:, [a, b]] for a, b in itertools.combinations(range(4), 2)])
        keys = pairs[:, 0] * nv + pairs[:, 1]
        ukeys, inv = np.unique(keys, return_inverse=True)
        self.edges = np.stack([ukeys // nv, ukeys % nv], axis=1)
        self.n_edges = self.edges.shape[0]
        nt = t.shape[0]
        # tet -> its 6 edge ids in the order (01,02,03,12,13,23)
        self.tet_edges = inv.reshape(6, nt).T.copy()
        # faces
        tri = np.concatenate([t[:, list(c)] for c in itertools.combinations(range(4), 3)])
        fkeys = (tri[:, 0] * nv + tri[:, 1]) * nv + tri[:, 2]
        ufk, fcount = np.unique(fkeys, return_counts=True)
        self.faces = np.stack([ufk // (nv * nv), (ufk // nv) % nv, ufk % nv], axis=1)
        bfaces = self.faces[fcount == 1]
        self.boundary_vertex = np.zeros(nv, dtype=bool)
        self.boundary_vertex[bfaces.ravel()] = True
        ekey = self.edges[:, 0] * nv + self.edges[:, 1]
        bpairs = np.concatenate([bfaces[:, [0, 1]], bfaces[:, [1, 2]], bfaces[:, [0, 2]]])
        bkeys = np.unique(bpairs[:, 0] * nv + bpairs[:, 1])
        self.boundary_edge = np.isin(ekey, bkeys)
        # free degrees of freedom ("interior" in the Dirichlet sense)
        if bc == DIRICHLET:
            self.interior_edges = np.flatnonzero(~self.boundary_edge)
            self.interior_vertices = np.flatnonzero(~self.boundary_vertex)
        else:
            self.interior_edges = np.arange(self.n_edges)
            self.interior_vertices = np.arange(1, nv)   # vertex 0 is the gauge vertex
        self._ekey_sorted = ekey  # sorted ascending by construction

    def edge_index(self, a, b):
        """Edge ids of vertex pairs (a, b) (either orientation); -1 if absent."""
        a = np.asarray(a, dtype=np.int64)
        b = np.asarray(b, dtype=np.int64)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        k = lo * self.n_vertices + hi
        pos = np.searchsorted(self._ekey_sorted, k)
        pos = np.minimum(pos, self.n_edges - 1)
        ok = self._ekey_sorted[pos] == k
        return np.where(ok, pos, -1)

    def gradient(self) -> sp.csr_matrix:
        """G (all edges x all vertices): +1 at head, -1 at tail."""
        E = self.n_edges
        rows = np.repeat(np.arange(E), 2)
        cols = self.edges[:, [1, 0]].ravel()
        vals = np.tile([1.0, -1.0], E)
        return sp.csr_matrix((vals, (rows, cols)), shape=(E, self.n_vertices))

    def curl(self) -> sp.csr_matrix:
        """C (all faces x all edges): +[a,b] + [b,c] - [a,c] for face a<b<c."""
        f = self.faces
        nf = f.shape[0]
        e_ab = self.edge_index(f[:, 0], f[:, 1])
        e_bc = self.edge_index(f[:, 1], f[:, 2])
        e_ac = self.edge_index(f[:, 0], f[:, 2])
        rows = np.repeat(np.arange(nf), 3)
        cols = np.stack([e_ab, e_bc, e_ac], axis=1).ravel()
        vals = np.tile([1.0, 1.0, -1.0], nf)
        return sp.csr_matrix((vals, (rows, cols)), shape=(nf, self.n_edges))

    def longest_edge(self) -> np.ndarray:
        """h_T: length of the longest edge of each tetrahedron (eq. (3))."""
        c = self.coords[self.tets]
        h = np.zeros(self.tets.shape[0])
        for a, b in itertools.combinations(range(4), 2):
            h = np.maximum(h, np.linalg.norm(c[:, a] - c[:, b], axis=1))
        return h

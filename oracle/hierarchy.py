"""Space-time level hierarchy, coarsening rule and transfers (oracle, test infrastructure).

* Time coarsening by a factor 2 down to one slab (the V-cycle over time meshes
  of section 2.1).
* Spatial coarsening only where the local degree of anisotropy of eq. (3),
  lambda(T) = min_{x in T} beta tau / (alpha h_T^2) with alpha = sigma,
  beta = nu = mu^{-1} and h_T the longest tetrahedron edge, is >= lambda_crit
  for every tetrahedron; lambda_crit = 0.1, the value section 5.1 finds for 3D
  lowest-order Nedelec elements with the SAS smoother. The finer level's tau
  and mesh decide whether the next coarser level also coarsens in space.
* Coarse spatial matrices are Galerkin products P_e^T M P_e and P_e^T K P_e
  with the Whitney edge prolongation P_e; the coarse nodal stiffness is
  G_c^T M_c G_c (the paper's K_n is the stiffness of div sigma grad, which
  equals G^T M G).
* Edge prolongation: a fine edge p->q inside a coarse tetrahedron takes
  lambda_i(p) lambda_j(q) - lambda_i(q) lambda_j(p) from the coarse edge i->j
  (the line integral of the coarse Whitney function along p->q). A fine vertex
  is a coarse vertex (lambda = 1) or the midpoint of a coarse edge (lambda =
  1/2 at both ends), which is all that nested refinement produces.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import DIRICHLET, Topology
from .fem import assemble_edge_matrices


class SpaceData:
    """Spatial operators of one mesh level restricted to interior DOFs."""

    def __init__(self, topo: Topology, M, K, ratio, Pe=None, Pn=None):
        self.topo = topo
        ie, iv = topo.interior_edges, topo.interior_vertices
        self.ie, self.iv = ie, iv
        self.n_e, self.n_v = ie.size, iv.size
        self.M = sp.csr_matrix(M)
        self.K = sp.csr_matrix(K)
        G = topo.gradient()
        self.G = sp.csr_matrix(G[ie][:, iv])
        self.Kn = sp.csr_matrix(self.G.T @ self.M @ self.G)
        self.ratio = ratio                  # nu/sigma per tet (min over children)
        self.h = topo.longest_edge()
        self.Pe = Pe                        # finer interior edges x these interior edges
        self.Pn = Pn                        # finer interior vertices x these interior vertices

    def anisotropy(self, tau: float) -> float:
        """lambda = min_T ratio_T tau / h_T^2 (eq. (3))."""
        return float(np.min(self.ratio * tau / self.h ** 2))


def edge_prolongation(fine: Topology, coarse: Topology, vertex_parent: np.ndarray) -> sp.csr_matrix:
    """P_e over ALL edges (fine edges x coarse edges), Whitney line integrals."""
    vp = np.asarray(vertex_parent, dtype=np.int64)
    rows, cols, vals = [], [], []
    for e in range(fine.n_edges):
        p, q = fine.edges[e]
        lp = {}
        for a in vp[p]:
            lp[int(a)] = lp.get(int(a), 0.0) + 0.5
        lq = {}
        for a in vp[q]:
            lq[int(a)] = lq.get(int(a), 0.0) + 0.5
        support = sorted(set(lp) | set(lq))
        for ii in range(len(support)):
            for jj in range(ii + 1, len(support)):
                i, j = support[ii], support[jj]
                c = lp.get(i, 0.0) * lq.get(j, 0.0) - lq.get(i, 0.0) * lp.get(j, 0.0)
                if c != 0.0:
                    ce = int(coarse.edge_index(i, j))
                    if ce < 0:
                        raise ValueError("fine edge not inside one coarse tetrahedron")
                    rows.append(e)
                    cols.append(ce)
                    vals.append(c)
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.n_edges, coarse.n_edges))


def vertex_prolongation(fine: Topology, coarse: Topology, vertex_parent: np.ndarray) -> sp.csr_matrix:
    """P_n over all vertices: P1 interpolation (fine vertex = mean of its parent pair)."""
    vp = np.asarray(vertex_parent, dtype=np.int64)
    nvf = fine.n_vertices
    rows = np.repeat(np.arange(nvf), 2)
    P = sp.csr_matrix((np.full(2 * nvf, 0.5), (rows, vp.ravel())), shape=(nvf, coarse.n_vertices))
    P.sum_duplicates()
    return P


def problem_bc(problem):
    """The problem's boundary condition (Dirichlet unless it names Neumann)."""
    return getattr(problem, "bc", DIRICHLET)


def finest_space(problem):
    """SpaceData of the problem's finest mesh alone (no coarse meshes)."""
    lev = problem.levels[0]
    topo0 = Topology(lev.coords, lev.tets, problem_bc(problem))
    M, K = assemble_edge_matrices(topo0, problem.sigma, problem.nu)
    ie = topo0.interior_edges
    return SpaceData(topo0, M[ie][:, ie], K[ie][:, ie], problem.nu / problem.sigma)


def build_space_levels(problem):
    """SpaceData for every mesh of the problem's nested hierarchy (finest first)."""
    levs = problem.levels
    bc = problem_bc(problem)
    topo0 = Topology(levs[0].coords, levs[0].tets, bc)
    M, K = assemble_edge_matrices(topo0, problem.sigma, problem.nu)
    ie, iv = topo0.interior_edges, topo0.interior_vertices
    out = [SpaceData(topo0, M[ie][:, ie], K[ie][:, ie], problem.nu / problem.sigma)]
    for j in range(1, len(levs)):
        fine = out[-1]
        topo = Topology(levs[j].coords, levs[j].tets, bc)
        Pe_all = edge_prolongation(fine.topo, topo, levs[j].vertex_parent)
        Pn_all = vertex_prolongation(fine.topo, topo, levs[j].vertex_parent)
        Pe = sp.csr_matrix(Pe_all[fine.ie][:, topo.interior_edges])
        Pn = sp.csr_matrix(Pn_all[fine.iv][:, topo.interior_vertices])
        Mc = Pe.T @ fine.M @ Pe
        Kc = Pe.T @ fine.K @ Pe
        ratio = np.full(topo.tets.shape[0], np.inf)
        np.minimum.at(ratio, np.asarray(levs[j].tet_parent, dtype=np.int64), fine.ratio)
        out.append(SpaceData(topo, Mc, Kc, ratio, Pe, Pn))
    return out


class LevelSpec:
    """One space-time level: spatial mesh index, slab count, step size."""

    def __init__(self, space: int, N: int, tau: float):
        self.space, self.N, self.tau = space, N, tau

    def __repr__(self):
        return f"LevelSpec(space={self.space}, N={self.N}, tau={self.tau:.6g})"


def build_level_specs(space_levels, T: float, Nt: int, lambda_crit: float = 0.1,
                      allow_space: bool = True):
    """Finest first. Halve N each level; coarsen space where eq. (3) holds."""
    if Nt < 1 or (Nt & (Nt - 1)) != 0:
        raise ValueError("Nt must be a power of two")
    specs = [LevelSpec(0, Nt, T / Nt)]
    while specs[-1].N > 1:
        cur = specs[-1]
        j = cur.space
        coarsen = (allow_space and j + 1 < len(space_levels)
                   and space_levels[j].anisotropy(cur.tau) >= lambda_crit)
        specs.append(LevelSpec(j + 1 if coarsen else j, cur.N // 2, 2.0 * cur.tau))
    return specs

"""Seeded synthetic inputs for the space-time multigrid solver.

This module produces problem *inputs* only: structured Kuhn tetrahedral
meshes of the unit cube (with their nested coarse meshes and the parent maps
that describe the nesting), piecewise-constant material fields, Gaussian
right-hand sides and request streams. It contains none of the method's
arithmetic (no element matrices, no time discretisation, no solver steps), so
both the CPU oracle and the GPU library may consume what it produces.

Mesh conventions
----------------
* Vertex (i, j, k), 0 <= i, j, k <= n, has id ``i + (n+1)*(j + (n+1)*k)`` and
  logical position (i, j, k)/n.
* Every hex [i,i+1]x[j,j+1]x[k,k+1] is split into the 6 Kuhn tetrahedra: for
  each permutation p of the axes, the path (0,0,0) -> e_p0 -> e_p0+e_p1 ->
  (1,1,1).  All hexes share the same main diagonal, so the mesh is conforming
  and uniform refinement n -> 2n is nested (Freudenthal subdivision).
* A coarse level (n/2) is described relative to its fine level by
  ``vertex_parent[v_fine] = (a, b)``: the fine vertex is the midpoint of the
  coarse vertices a and b (a == b when it coincides with a coarse vertex), and
  ``tet_parent[t_fine]``: the coarse tetrahedron that contains the fine one.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# The six axis permutations in a fixed order; tet index inside a hex is the
# position of its permutation in this list.
KUHN_PERMS = list(itertools.permutations(range(3)))


def vertex_id(i, j, k, n):
    return i + (n + 1) * (j + (n + 1) * k)


def kuhn_tets(n: int) -> np.ndarray:
    """[6 n^3, 4] int32 tetrahedra of the Kuhn subdivision of an n^3 grid."""
    idx = np.arange(n)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    # hex order: i fastest, then j, then k (matches vertex numbering)
    I = I.transpose(2, 1, 0).ravel()
    J = J.transpose(2, 1, 0).ravel()
    K = K.transpose(2, 1, 0).ravel()
    base = np.stack([I, J, K], axis=1)  # [n^3, 3]
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for t, perm in enumerate(KUHN_PERMS):
        p = base.copy()
        tets[:, t, 0] = vertex_id(p[:, 0], p[:, 1], p[:, 2], n)
        for s in range(3):
            p[:, perm[s]] += 1
            tets[:, t, s + 1] = vertex_id(p[:, 0], p[:, 1], p[:, 2], n)
    return tets.reshape(-1, 4).astype(np.int32)


def kuhn_coords(n: int) -> np.ndarray:
    """[(n+1)^3, 3] float64 logical vertex positions (i, j, k)/n."""
    r = np.arange(n + 1, dtype=np.float64) / n
    K, J, I = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)


def jitter_coords(coords: np.ndarray, n: int, frac: float, rng) -> np.ndarray:
    """Shift every interior vertex coordinate independently by U[-frac*h, frac*h]."""
    out = coords.copy()
    h = 1.0 / n
    interior = np.all((coords > 0.5 * h) & (coords < 1.0 - 0.5 * h), axis=1)
    shift = rng.uniform(-frac * h, frac * h, size=(int(interior.sum()), 3))
    out[interior] += shift
    return out


@dataclass
class SpaceLevel:
    """One mesh of a nested hierarchy (finest first)."""
    n: int
    coords: np.ndarray          # [nv, 3] float64
    tets: np.ndarray            # [nt, 4] int32
    # Maps from the next finer level onto this one (None on the finest level).
    vertex_parent: np.ndarray | None = None   # [nv_finer, 2] int32
    tet_parent: np.ndarray | None = None      # [nt_finer] int32


@dataclass
class Problem:
    """Everything the solver is given: meshes, materials, time grid."""
    levels: list                 # list[SpaceLevel], finest first
    sigma: np.ndarray            # [nt_finest] float64
    nu: np.ndarray               # [nt_finest] float64
    T: float
    Nt: int
    pt: int
    meta: dict = field(default_factory=dict)
    # "dirichlet" (u x n = 0) or "neumann" (nu curl u x n = 0)
    bc: str = "dirichlet"

    @property
    def fine(self) -> SpaceLevel:
        return self.levels[0]


def _coarse_maps(n_fine: int):
    """vertex_parent and tet_parent from the Kuhn n_fine mesh to n_fine/2."""
    nc = n_fine // 2
    r = np.arange(n_fine + 1)
    K, J, I = np.meshgrid(r, r, r, indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    a = vertex_id(I // 2, J // 2, K // 2, nc)
    b = vertex_id((I + 1) // 2, (J + 1) // 2, (K + 1) // 2, nc)
    vparent = np.stack([a, b], axis=1).astype(np.int32)

    # tet_parent: the coarse Kuhn tet containing the centroid of each fine tet.
    ft = kuhn_tets(n_fine)
    fc = kuhn_coords(n_fine) * n_fine / 2.0  # fine vertices in coarse grid units
    cent = fc[ft].mean(axis=1)               # [nt, 3]
    hexc = np.floor(cent).astype(np.int64)
    loc = cent - hexc
    # Kuhn tet with permutation p holds points with loc[p0] >= loc[p1] >= loc[p2]
    order = np.argsort(-loc, axis=1, kind="stable")
    perm_index = {p: t for t, p in enumerate(KUHN_PERMS)}
    tidx = np.array([perm_index[tuple(o)] for o in order], dtype=np.int64)
    hid = hexc[:, 0] + nc * (hexc[:, 1] + nc * hexc[:, 2])
    tparent = (hid * 6 + tidx).astype(np.int32)
    return vparent, tparent


def kuhn_hierarchy(n: int, n_min: int = 2, jitter: float = 0.0, seed: int = 0):
    """Nested Kuhn meshes n, n/2, ..., down to n_min (finest first).

    With jitter > 0 the interior vertices of the finest mesh are shifted; each
    coarse mesh then takes the (shifted) positions of the fine vertices it
    shares, so coarse tetrahedra have the fine mesh's geometry at their corners.
    """
    rng = np.random.default_rng(seed)
    coords = kuhn_coords(n)
    if jitter > 0:
        coords = jitter_coords(coords, n, jitter, rng)
    levels = [SpaceLevel(n=n, coords=coords, tets=kuhn_tets(n))]
    m = n
    while m % 2 == 0 and m // 2 >= n_min:
        vp, tp = _coarse_maps(m)
        mc = m // 2
        fine_coords = levels[-1].coords
        # coarse vertex (i,j,k) is fine vertex (2i,2j,2k)
        r = np.arange(mc + 1)
        K, J, I = np.meshgrid(r, r, r, indexing="ij")
        src = vertex_id(2 * I.ravel(), 2 * J.ravel(), 2 * K.ravel(), m)
        levels.append(SpaceLevel(n=mc, coords=fine_coords[src].copy(), tets=kuhn_tets(mc),
                                 vertex_parent=vp, tet_parent=tp))
        m = mc
    return levels


# ---------------------------------------------------------------- materials
def block_materials(n: int, nblocks: int, sigma_range, nu_range, seed: int):
    """Piecewise-constant log-uniform sigma, nu on nblocks^3 blocks of hexes."""
    rng = np.random.default_rng(seed)
    nb = nblocks ** 3
    ls = rng.uniform(np.log10(sigma_range[0]), np.log10(sigma_range[1]), size=nb)
    ln = rng.uniform(np.log10(nu_range[0]), np.log10(nu_range[1]), size=nb)
    bs = n // nblocks
    hexes = np.arange(n ** 3)
    hi, hj, hk = hexes % n, (hexes // n) % n, hexes // (n * n)
    blk = (hi // bs) + nblocks * ((hj // bs) + nblocks * (hk // bs))
    blk_t = np.repeat(blk, 6)
    return 10.0 ** ls[blk_t], 10.0 ** ln[blk_t]


def core_box_materials(coords, tets, lo=0.3, hi=0.7, sigma_in=1e4, sigma_out=1e-2,
                       nu_in=1e-3, nu_out=1.0):
    """High-contrast conducting core: a tet is in the core iff its centroid is."""
    cent = coords[tets].mean(axis=1)
    inside = np.all((cent > lo) & (cent < hi), axis=1)
    sigma = np.where(inside, sigma_in, sigma_out).astype(np.float64)
    nu = np.where(inside, nu_in, nu_out).astype(np.float64)
    return sigma, nu


def gaussian_rhs(n_edges: int, Nt: int, pt: int, seed: int) -> np.ndarray:
    """[Nt, pt+1, n_edges] float64 standard normal load vector."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((Nt, pt + 1, n_edges))


def count_edges(tets: np.ndarray, n_vertices: int) -> int:
    """Number of distinct mesh edges (topology bookkeeping for sizing inputs)."""
    t = tets.astype(np.int64)
    pairs = np.concatenate([np.sort(t[:, [a, b]], axis=1)
                            for a, b in itertools.combinations(range(4), 2)])
    return int(np.unique(pairs[:, 0] * n_vertices + pairs[:, 1]).size)


# -------------------------------------------------------------- workloads
def config_unit_manufactured(n: int = 4, Nt: int = 16, pt: int = 1, T: float = 1.0) -> Problem:
    """sigma = nu = 1 on the n^3 Kuhn cube (rhs comes from the manufactured field)."""
    levels = kuhn_hierarchy(n)
    nt = levels[0].tets.shape[0]
    return Problem(levels, np.ones(nt), np.ones(nt), T, Nt, pt,
                   meta={"name": f"manufactured n={n} Nt={Nt} pt={pt}"})


def config_block_random(n: int = 32, Nt: int = 256, pt: int = 1, T: float = 1.0,
                        seed: int = 1, block_hexes: int = 8,
                        sigma_range=(1.0, 1e3), nu_range=(1.0, 100.0)) -> Problem:
    """Block-constant log-uniform materials on block_hexes^3 blocks."""
    levels = kuhn_hierarchy(n)
    nblocks = max(1, n // block_hexes)
    sigma, nu = block_materials(n, nblocks, sigma_range, nu_range, seed)
    return Problem(levels, sigma, nu, T, Nt, pt,
                   meta={"name": f"block-random n={n} Nt={Nt} pt={pt} seed={seed}"})


def config_core_box(n: int = 64, Nt: int = 128, pt: int = 1, T: float = 1.0,
                    seed: int = 3, jitter: float = 0.2) -> Problem:
    """Jittered mesh with a high-contrast conducting core box [0.3, 0.7]^3."""
    levels = kuhn_hierarchy(n, jitter=jitter, seed=seed)
    sigma, nu = core_box_materials(levels[0].coords, levels[0].tets)
    return Problem(levels, sigma, nu, T, Nt, pt,
                   meta={"name": f"jittered core-box n={n} Nt={Nt} pt={pt} seed={seed}"})


def request_stream(n_requests: int = 512, rate: float = 1.0, seed: int = 5,
                   sizes=(8, 12, 16, 24, 32), horizons=(16, 64, 128, 256, 512),
                   degrees=(0, 1)):
    """Poisson arrivals of solve requests: (arrival_time, n, Nt, pt, seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    out = []
    for r in range(n_requests):
        out.append(dict(arrival=float(t[r]), n=int(rng.choice(sizes)),
                        Nt=int(rng.choice(horizons)), pt=int(rng.choice(degrees)),
                        seed=int(1000 + r)))
    return out


def config_request(n: int, Nt: int, pt: int, seed: int, T: float = 1.0) -> Problem:
    """One serving request: block-random sigma in [1e-2,1e4], nu in [1e-3,100]."""
    levels = kuhn_hierarchy(n)
    nblocks = 4 if n % 4 == 0 else 1
    sigma, nu = block_materials(n, nblocks, (1e-2, 1e4), (1e-3, 100.0), seed)
    return Problem(levels, sigma, nu, T, Nt, pt, meta={"name": f"request n={n} Nt={Nt} pt={pt}"})


def config_two_lambda(n: int, Nt: int, pt: int, T: float, nu2: float, n_meshes: int = 2) -> Problem:
    """Two materials with different anisotropy (the "Two lambda" case): the
    cube's halves x < 1/2 (nu = 1) and x > 1/2 (nu = nu2 >= 1) by tet
    centroid, sigma = 1, Neumann boundary, the n^3 Kuhn mesh and its next
    n_meshes - 1 coarser meshes."""
    levels = kuhn_hierarchy(n)[:n_meshes]
    fine = levels[0]
    cx = fine.coords[fine.tets][:, :, 0].mean(axis=1)
    nt = fine.tets.shape[0]
    nu = np.where(cx > 0.5, float(nu2), 1.0)
    return Problem(levels, np.ones(nt), nu, T, Nt, pt, bc="neumann",
                   meta={"name": f"two-lambda n={n} Nt={Nt} pt={pt} T={T} nu2={nu2}"})

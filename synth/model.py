"""Seeded tight-binding model generator (input data for every test and benchmark).

The paper's workloads are SCC-DFTB Hamiltonians of solvated polyalanine and liquid
water in a local basis (Results section).  Neither structure nor the DFTB
parameters are available, so a random geometric two-orbital tight-binding model
with the same character stands in: sparse, symmetric, local, gapped.

Every floating-point value is produced with IEEE-754 basic operations only
(+, -, *, /, sqrt, rint, ldexp), so the arrays are bit-identical on every
machine; the exponential used by the hopping is evaluated by a fixed polynomial
below rather than by the platform's libm.

Model (all lengths in Angstrom, energies in eV):
  * sites uniform in a periodic cube of side L = (n_sites / density)^(1/3)
    (or clustered, see ``clustered_sites``), sorted by a 30-bit Morton code so
    that vertex order is spatially local;
  * two orbitals per site, orbital index 2*site + a;
  * onsite energy -1.5 (a = 0) or +1.5 (a = 1) plus U(-0.1, 0.1) noise drawn
    after sorting, in orbital order;
  * hopping t(r) = -0.3 exp(-r / 1.5) between every orbital pair of two
    distinct sites closer than 6 (minimum image); the same-site off-diagonal
    element is 0.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CONFIGS", "ModelSpec", "make_model", "make_operator_v", "operator_v_pairs", "displace_sites",
    "rebuild_hamiltonian", "ell_sha256", "det_exp",
]


@dataclass(frozen=True)
class ModelSpec:
    """Parameters of one synthetic system."""
    n_sites: int
    density: float = 0.1            # sites per cubic Angstrom
    seed: int = 0
    onsite: tuple = (-1.5, 1.5)     # per orbital kind a = 0, 1
    noise: float = 0.1              # onsite noise half-width
    t0: float = -0.3                # hopping prefactor
    decay: float = 1.5              # hopping decay length
    cutoff: float = 6.0             # hopping range
    clusters: tuple = ()            # (n_spheres, sites_per_sphere, dense_density) or ()
    name: str = field(default="", compare=False)


# The five workloads: N = 1024 (FP64 reference size), N = 18000 (batched), the
# heterogeneous N = 100000 system (70 % of sites in dense spheres), and small
# systems for brute-force checks.
CONFIGS = {
    "n1024": ModelSpec(n_sites=512, seed=1, name="n1024"),
    "n18000": ModelSpec(n_sites=9000, seed=2, name="n18000"),
    "n100000": ModelSpec(n_sites=50000, seed=4, clusters=(70, 500, 0.15), density=0.03,
                         name="n100000"),
    # brute-force scale: low density so that the periodic box exceeds twice the cutoff
    "tiny48": ModelSpec(n_sites=24, density=0.01, seed=7, cutoff=6.0, name="tiny48"),
    "small256": ModelSpec(n_sites=128, density=0.05, seed=3, name="small256"),
    "n4096": ModelSpec(n_sites=2048, seed=5, name="n4096"),
    # beyond the n-bit LDS bitmaps of the graph and halo kernels (their hash-set paths)
    "n500000": ModelSpec(n_sites=250000, seed=6, name="n500000"),
}

_LN2_HI = 6.93147180369123816490e-01   # ln 2 high part, low bits zero
_LN2_LO = 1.90821492927058770002e-10   # ln 2 - _LN2_HI
_INV_LN2 = 1.44269504088896338700e+00


def det_exp(x: np.ndarray) -> np.ndarray:
    """exp(x) for moderate |x| from basic IEEE operations only (bit-reproducible).

    Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2, then the degree-17 Taylor
    polynomial of exp(r) in Horner form (truncation < 1e-19 relative) and an exact
    scaling by 2^k.
    """
    x = np.asarray(x, dtype=np.float64)
    k = np.rint(x * _INV_LN2)
    r = (x - k * _LN2_HI) - k * _LN2_LO
    p = np.ones_like(r)
    for n in range(17, 0, -1):
        p = 1.0 + (r / float(n)) * p
    return np.ldexp(p, k.astype(np.int64))


def _box_length(volume: float) -> float:
    # the cube root is rounded to 1e-9 so that the box side does not depend on libm
    return float(round(volume ** (1.0 / 3.0), 9))


def _wrap(pos: np.ndarray, L: float) -> np.ndarray:
    pos = pos - L * np.floor(pos / L)
    return np.where(pos >= L, pos - L, pos)


def clustered_sites(rng: np.random.Generator, n_spheres: int, per_sphere: int,
                    dense_density: float, n_dilute: int, dilute_density: float):
    """Heterogeneous geometry: dense spheres in a dilute background.

    Sphere radius R = (3 per_sphere / (4 pi dense_density))^(1/3); centres are placed
    by random sequential addition with minimum-image separation > 2R; sphere sites are
    uniform in the ball (rejection from its bounding cube); dilute sites are uniform in
    the box and rejected if they fall inside any sphere.  The box volume is the sum of
    the sphere volumes and the dilute volume n_dilute / dilute_density.
    """
    sphere_vol = per_sphere / dense_density
    R = float(round((3.0 * sphere_vol / (4.0 * np.pi)) ** (1.0 / 3.0), 9))
    L = _box_length(n_spheres * sphere_vol + n_dilute / dilute_density)
    centres = np.zeros((0, 3))
    while centres.shape[0] < n_spheres:
        c = rng.uniform(0.0, L, 3)
        if centres.shape[0]:
            d = centres - c
            d = d - L * np.rint(d / L)
            d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            if np.any(d2 <= (2.0 * R) * (2.0 * R)):
                continue
        centres = np.vstack([centres, c])
    pts = []
    for c in centres:
        got = np.zeros((0, 3))
        while got.shape[0] < per_sphere:
            u = rng.uniform(-R, R, (2 * per_sphere, 3))
            u2 = (u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1]) + u[:, 2] * u[:, 2]
            got = np.vstack([got, u[u2 < R * R]])
        pts.append(_wrap(got[:per_sphere] + c, L))
    dil = np.zeros((0, 3))
    while dil.shape[0] < n_dilute:
        u = rng.uniform(0.0, L, (n_dilute, 3))
        inside = np.zeros(u.shape[0], dtype=bool)
        for c in centres:
            d = u - c
            d = d - L * np.rint(d / L)
            d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            inside |= d2 < R * R
        dil = np.vstack([dil, u[~inside]])
    pts.append(dil[:n_dilute])
    return np.vstack(pts), L


def morton_order(pos: np.ndarray, L: float) -> np.ndarray:
    """Stable argsort by the 30-bit Morton code of the positions (10 bits per axis)."""
    q = np.minimum(np.floor(pos / L * 1024.0).astype(np.int64), 1023)
    code = np.zeros(pos.shape[0], dtype=np.int64)
    for b in range(10):
        for d in range(3):
            code |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return np.argsort(code, kind="stable")


def _site_pairs(pos: np.ndarray, L: float, cutoff: float):
    """Unordered site pairs (i < j) with minimum-image distance < cutoff, and r."""
    from scipy.spatial import cKDTree  # candidate search only; r is recomputed below

    tree = cKDTree(pos, boxsize=L)
    pairs = tree.query_pairs(r=cutoff + 1e-6, output_type="ndarray")
    if pairs.size == 0:
        return np.zeros((0, 2), dtype=np.int64), np.zeros(0)
    pairs = np.sort(pairs.astype(np.int64), axis=1)
    d = pos[pairs[:, 1]] - pos[pairs[:, 0]]
    d = d - L * np.rint(d / L)
    r = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    keep = r < cutoff
    return pairs[keep], r[keep]


def _hamiltonian_ell(pos: np.ndarray, L: float, onsite_vals: np.ndarray, spec: ModelSpec):
    n_sites = pos.shape[0]
    N = 2 * n_sites
    pairs, r = _site_pairs(pos, L, spec.cutoff)
    t = spec.t0 * det_exp(-(r / spec.decay))
    rows = [np.arange(N, dtype=np.int64)]
    cols = [np.arange(N, dtype=np.int64)]
    vals = [onsite_vals]
    for a in (0, 1):
        for b in (0, 1):
            ri = 2 * pairs[:, 0] + a
            cj = 2 * pairs[:, 1] + b
            rows += [ri, cj]
            cols += [cj, ri]
            vals += [t, t]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=N)
    W = int(counts.max())
    start = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=start[1:])
    slot = np.arange(rows.size, dtype=np.int64) - start[rows]
    col = np.full((N, W), -1, dtype=np.int32)
    val = np.zeros((N, W), dtype=np.float64)
    col[rows, slot] = cols.astype(np.int32)
    val[rows, slot] = vals
    return col, val


def _onsite(rng: np.random.Generator, n_sites: int, spec: ModelSpec) -> np.ndarray:
    base = np.tile(np.asarray(spec.onsite, dtype=np.float64), n_sites)
    return base + rng.uniform(-spec.noise, spec.noise, 2 * n_sites)


def make_model(spec, seed: int | None = None) -> dict:
    """Build the seeded system for ``spec`` (a ModelSpec or a key of CONFIGS).

    Returns a dict with the ELL arrays ``H_col`` (int32 [N, W], ascending columns,
    padding -1) and ``H_val`` (float64 [N, W], padding 0), ``N``, ``n_occ`` = N/2,
    ``pos`` (Morton-sorted site positions), ``L`` and ``onsite``.
    """
    if isinstance(spec, str):
        spec = CONFIGS[spec]
    if seed is None:
        seed = spec.seed
    rng = np.random.default_rng(seed)
    if spec.clusters:
        n_sph, per, rho = spec.clusters
        n_dil = spec.n_sites - n_sph * per
        pos, L = clustered_sites(rng, n_sph, per, rho, n_dil, spec.density)
    else:
        L = _box_length(spec.n_sites / spec.density)
        pos = rng.uniform(0.0, L, (spec.n_sites, 3))
    if L <= 2.0 * spec.cutoff:
        raise ValueError("periodic box must exceed twice the hopping cutoff")
    pos = pos[morton_order(pos, L)]
    onsite = _onsite(rng, spec.n_sites, spec)
    col, val = _hamiltonian_ell(pos, L, onsite, spec)
    N = 2 * spec.n_sites
    return {"H_col": col, "H_val": val, "N": N, "n_occ": N // 2, "pos": pos, "L": L,
            "onsite": onsite, "spec": spec, "seed": seed}


def rebuild_hamiltonian(model: dict, pos: np.ndarray) -> dict:
    """Same system (same onsite energies, same site order) at new positions."""
    spec = model["spec"]
    col, val = _hamiltonian_ell(pos, model["L"], model["onsite"], spec)
    out = dict(model)
    out.update(H_col=col, H_val=val, pos=pos)
    return out


def displace_sites(pos: np.ndarray, L: float, sigma: float, rng: np.random.Generator):
    """Gaussian displacement of every coordinate, wrapped back into the box."""
    return _wrap(pos + rng.normal(0.0, sigma, pos.shape), L)


def make_operator_v(H_col: np.ndarray, seed: int) -> np.ndarray:
    """A random symmetric operator V on H's pattern: U(-1, 1) drawn for the upper
    triangle (including the diagonal) in ELL row-major order, mirrored below."""
    N, W = H_col.shape
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(N), W).reshape(N, W)
    upper = (H_col >= 0) & (H_col >= rows)
    draws = rng.uniform(-1.0, 1.0, int(upper.sum()))
    V = np.zeros(H_col.shape, dtype=np.float64)
    V[upper] = draws
    # mirror: entry (i, j) with j < i takes the value of (j, i)
    lower = (H_col >= 0) & (H_col < rows)
    li, ls = np.nonzero(lower)
    lj = H_col[li, ls].astype(np.int64)
    # position of column i in row j
    pos_in_row = np.array([np.searchsorted(H_col[j][H_col[j] >= 0], i) for i, j in zip(li, lj)],
                          dtype=np.int64) if li.size < 200000 else _bulk_find(H_col, lj, li)
    V[li, ls] = V[lj, pos_in_row]
    return V


def operator_v_pairs(H_col: np.ndarray, seed: int) -> np.ndarray:
    """A symmetric operator V on H's pattern whose entry for the orbital pair {i, j} does not
    depend on the pattern: U(-1, 1) from a SplitMix64 hash of (seed, min(i, j), max(i, j)).  Used
    where the pattern changes between uses (displacement steps) and V must stay the same."""
    N, W = H_col.shape
    rows = np.repeat(np.arange(N, dtype=np.uint64), W).reshape(N, W)
    cols = np.where(H_col >= 0, H_col, 0).astype(np.uint64)
    a = np.minimum(rows, cols)
    b = np.maximum(rows, cols)
    with np.errstate(over="ignore"):
        z = (np.uint64(seed) * np.uint64(0x9E3779B97F4A7C15) + a * np.uint64(1 << 32) + b)
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)  # [0, 1)
    return np.where(H_col >= 0, 2.0 * u - 1.0, 0.0)


def _bulk_find(H_col, rows, targets):
    """Slot of column ``targets[k]`` in ELL row ``rows[k]`` (vectorised)."""
    N, W = H_col.shape
    key = np.where(H_col >= 0, H_col, np.iinfo(np.int32).max).astype(np.int64)
    flat = (np.arange(N, dtype=np.int64)[:, None] * (1 << 32) + key).ravel()
    q = rows.astype(np.int64) * (1 << 32) + targets.astype(np.int64)
    idx = np.searchsorted(flat, q)
    return (idx - rows.astype(np.int64) * W).astype(np.int64)


def ell_sha256(*arrays) -> str:
    """SHA-256 over the raw little-endian bytes of the given arrays."""
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()

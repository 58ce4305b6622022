"""Seeded synthetic workloads for pass-through connectivity counting.

This module only *draws inputs*: streamlines (random walks in voxel
coordinates), an ROI index volume and a target label volume.  It contains no
part of the counting method (no voxelisation of streamline points, no set or
matrix arithmetic) and serves the HIP path, the CPU oracle, the tests and the
benchmark alike.

The paper's own data (HCP subjects tracked with MRtrix3, thalamus ROI and
Desikan-Killiany targets; Section 3) are not available, so these recipes stand
in for them with the same structure: a compact seed ROI whose voxels are rows
0..N-1 in raster order, M target labels tiling a thin cortical shell, and
probabilistic-tractography-like walks with a 0.5-voxel step.

Coordinates are voxel coordinates with voxel centres at integers.  Volumes are
numpy/torch arrays shaped [Z, Y, X] (x fastest).  Walks are drawn with torch's
Philox generator on the requested device, chunk by chunk (2^18 streamlines per
chunk, seeded from (seed, chunk)), so a (seed, device) pair fixes every value;
CPU and GPU draws differ from each other.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence, Tuple

import numpy as np
import torch

CHUNK = 1 << 18          # streamlines per generator chunk (fixed: part of the recipe)
STEP = 0.5               # walk step, voxels
SIGMA = 0.15             # per-step direction perturbation (std of each Gaussian component)
SR_SCALE = float(np.float32(1.25 / 0.7))   # 1.25 mm grid -> 0.7 mm grid, fl32 = 1.7857143


@dataclasses.dataclass
class Volumes:
    roi: np.ndarray          # [Z,Y,X] int32, row index in [0,N) or -1
    lab: np.ndarray          # [Z,Y,X] int32, label in [0,M) or -1
    N: int
    M: int
    centre: Tuple[float, float, float]
    brain_semi: Optional[Tuple[float, float, float]]   # mask ellipsoid (None: no mask stop)
    roi_ellipsoids: Sequence[Tuple[Tuple[float, float, float], Tuple[float, float, float]]]

    @property
    def dims(self) -> Tuple[int, int, int]:
        Z, Y, X = self.roi.shape
        return (X, Y, Z)


@dataclasses.dataclass
class Workload:
    name: str
    points: torch.Tensor     # [P,3] float32
    offsets: torch.Tensor    # [S+1] int64
    roi: torch.Tensor        # [Z,Y,X] int32
    lab: torch.Tensor        # [Z,Y,X] int32
    N: int
    M: int
    scale: float = 1.0

    @property
    def dims(self) -> Tuple[int, int, int]:
        Z, Y, X = self.roi.shape
        return (int(X), int(Y), int(Z))

    @property
    def S(self) -> int:
        return int(self.offsets.shape[0]) - 1

    @property
    def P(self) -> int:
        return int(self.points.shape[0])

    def to(self, device) -> "Workload":
        return dataclasses.replace(self, points=self.points.to(device), offsets=self.offsets.to(device),
                                   roi=self.roi.to(device), lab=self.lab.to(device))


# ----------------------------------------------------------------------------------------------
# volumes (numpy, deterministic on every machine)
# ----------------------------------------------------------------------------------------------

def _grid(dims):
    X, Y, Z = dims
    z = np.arange(Z, dtype=np.float64)[:, None, None]
    y = np.arange(Y, dtype=np.float64)[None, :, None]
    x = np.arange(X, dtype=np.float64)[None, None, :]
    return x, y, z


def ellipsoid(dims, centre, semi) -> np.ndarray:
    """Voxels (integer centres) inside a closed axis-aligned ellipsoid, [Z,Y,X] bool."""
    x, y, z = _grid(dims)
    cx, cy, cz = centre
    ax, ay, az = semi
    return ((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 + ((z - cz) / az) ** 2 <= 1.0


def index_in_raster_order(mask: np.ndarray) -> Tuple[np.ndarray, int]:
    """ROI index volume: masked voxels numbered 0..N-1 in raster order (x fastest), else -1."""
    roi = np.full(mask.shape, -1, dtype=np.int32)
    flat = np.flatnonzero(mask.reshape(-1))
    roi.reshape(-1)[flat] = np.arange(flat.size, dtype=np.int32)
    return roi, int(flat.size)


def nearest_centroid_labels(shell: np.ndarray, M: int, rng: np.random.Generator) -> np.ndarray:
    """Label volume: M centroids drawn from the shell voxels; each shell voxel takes the
    nearest centroid's label (ties -> lower label); voxels off the shell get -1."""
    lab = np.full(shell.shape, -1, dtype=np.int32)
    zyx = np.argwhere(shell)                         # raster order
    pick = rng.choice(zyx.shape[0], size=M, replace=False)
    cent = zyx[pick].astype(np.int64)
    out = np.empty(zyx.shape[0], dtype=np.int32)
    step = 1 << 16
    for a in range(0, zyx.shape[0], step):
        v = zyx[a:a + step].astype(np.int64)
        d2 = ((v[:, None, :] - cent[None, :, :]) ** 2).sum(-1)      # exact integers
        out[a:a + step] = np.argmin(d2, axis=1)                        # first minimum
    lab[shell] = out
    return lab


CFG2_DIMS = (145, 174, 145)
CFG2_CENTRE = (72.0, 87.0, 72.0)
CFG2_BRAIN = (56.0, 68.0, 52.0)
CFG2_ROI_SEMI = (8.0, 12.0, 10.0)
CFG2_ROI_CENTRES = ((61.0, 82.0, 77.0), (83.0, 82.0, 77.0))


def volumes_tiny64() -> Volumes:
    """64^3 grid: ellipsoid ROI (semi-axes 10,8,7 at the centre), M=8 octant labels on the
    shell 26 <= |v - c| <= 30."""
    dims = (64, 64, 64)
    c = (32.0, 32.0, 32.0)
    roi, N = index_in_raster_order(ellipsoid(dims, c, (10.0, 8.0, 7.0)))
    Z, Y, X = 64, 64, 64
    z = np.arange(Z)[:, None, None]
    y = np.arange(Y)[None, :, None]
    x = np.arange(X)[None, None, :]
    d2 = (x - 32) ** 2 + (y - 32) ** 2 + (z - 32) ** 2
    shell = (d2 >= 26 * 26) & (d2 <= 30 * 30)
    octant = (4 * (x >= 32) + 2 * (y >= 32) + (z >= 32)).astype(np.int32)
    lab = np.where(shell, np.broadcast_to(octant, shell.shape), -1).astype(np.int32)
    return Volumes(roi, lab, N, 8, c, None, [(c, (10.0, 8.0, 7.0))])


def volumes_interleaved64() -> Volumes:
    """64^3 grid where ROI and labels alternate in 4-voxel cubes inside a ball of radius 30: the
    cubes with an even (x//4 + y//4 + z//4) are ROI voxels, the odd ones carry one of M=8 labels,
    (x//4 + 2 (y//4) + 4 (z//4)) mod 8.  A walk of a few points already crosses both, so short
    streamlines produce pairs (unlike the shell layout, where ROI and labels are 16 voxels apart)."""
    dims = (64, 64, 64)
    c = (32.0, 32.0, 32.0)
    ball = ellipsoid(dims, c, (30.0, 30.0, 30.0))
    z = np.arange(64)[:, None, None] // 4
    y = np.arange(64)[None, :, None] // 4
    x = np.arange(64)[None, None, :] // 4
    even = ((x + y + z) % 2 == 0)
    roi, N = index_in_raster_order(ball & even)
    code = ((x + 2 * y + 4 * z) % 8).astype(np.int32)
    lab = np.where(ball & ~even, np.broadcast_to(code, ball.shape), -1).astype(np.int32)
    return Volumes(roi, lab, N, 8, c, None, [(c, (30.0, 30.0, 30.0))])


def volumes_subject(dims, centre, brain, roi_semi, roi_centres, M: int, shell_thickness: float,
                    rng: np.random.Generator) -> Volumes:
    """Ellipsoidal brain mask, two ROI ellipsoids (bilateral seed ROI), and M labels tiling the
    outer shell of the mask (mask minus the mask shrunk by ``shell_thickness`` voxels)."""
    mask = ellipsoid(dims, centre, brain)
    inner = ellipsoid(dims, centre, tuple(a - shell_thickness for a in brain))
    shell = mask & ~inner
    roi_mask = np.zeros_like(mask)
    for rc in roi_centres:
        roi_mask |= ellipsoid(dims, rc, roi_semi)
    roi_mask &= ~shell
    roi, N = index_in_raster_order(roi_mask)
    lab = nearest_centroid_labels(shell, M, rng)
    return Volumes(roi, lab, N, M, tuple(centre), tuple(brain),
                   [(tuple(rc), tuple(roi_semi)) for rc in roi_centres])


def volumes_125mm(seed: int = 2) -> Volumes:
    """145x174x145 grid, bilateral ROI (about 8k voxels), M=70 labels on a 3-voxel shell."""
    return volumes_subject(CFG2_DIMS, CFG2_CENTRE, CFG2_BRAIN, CFG2_ROI_SEMI, CFG2_ROI_CENTRES,
                           70, 3.0, np.random.default_rng([seed, 0]))


def volumes_07mm(seed: int = 3) -> Volumes:
    """260x311x260 grid: the 1.25 mm anatomy scaled by 1.25/0.7 (ROI about 45.8k voxels),
    M=180 labels on a 3-voxel shell."""
    s = 1.25 / 0.7
    sc = lambda v: tuple(float(a) * s for a in v)   # noqa: E731
    return volumes_subject((260, 311, 260), sc(CFG2_CENTRE), sc(CFG2_BRAIN), sc(CFG2_ROI_SEMI),
                           [sc(c) for c in CFG2_ROI_CENTRES], 180, 3.0, np.random.default_rng([seed, 0]))


# ----------------------------------------------------------------------------------------------
# walks (torch, chunked, on any device)
# ----------------------------------------------------------------------------------------------

def _chunk_generator(seed: int, chunk: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1_000_003 + int(chunk) * 7919 + 12345) % (2 ** 63 - 1))
    return g


def _unit(v: torch.Tensor) -> torch.Tensor:
    return v / torch.linalg.vector_norm(v, dim=-1, keepdim=True)


def uniform_in_ellipsoid(n, centre, semi, g, device) -> torch.Tensor:
    d = _unit(torch.randn(n, 3, generator=g, device=device, dtype=torch.float64))
    r = torch.rand(n, 1, generator=g, device=device, dtype=torch.float64) ** (1.0 / 3.0)
    return torch.tensor(centre, dtype=torch.float64, device=device) + \
        d * r * torch.tensor(semi, dtype=torch.float64, device=device)


def random_walks(n: int, seeds: torch.Tensor, lengths: torch.Tensor, g: torch.Generator,
                 inside: Optional[Callable[[torch.Tensor], torch.Tensor]] = None):
    """Walks p_0 = seed, d_0 uniform on the sphere, d <- normalize(d + SIGMA*N(0,I)),
    p <- p + STEP*d, in float64; a walk ends after ``lengths`` points or, when ``inside`` is
    given, at its first step outside (that point is not kept).  Returns points [P,3] float32
    (streamline-major) and per-walk point counts [n] int64."""
    device = seeds.device
    Tmax = int(lengths.max().item()) if n else 0
    buf = torch.empty((n, max(Tmax, 1), 3), dtype=torch.float32, device=device)
    p = seeds.clone()
    d = _unit(torch.randn(n, 3, generator=g, device=device, dtype=torch.float64))
    buf[:, 0] = p.float()
    alive = torch.ones(n, dtype=torch.bool, device=device)
    L = torch.ones(n, dtype=torch.int64, device=device)
    for t in range(1, Tmax):
        alive &= lengths > t
        if t % 32 == 0 and not bool(alive.any()):
            break
        d = _unit(d + SIGMA * torch.randn(n, 3, generator=g, device=device, dtype=torch.float64))
        p = p + STEP * d
        if inside is not None:
            alive &= inside(p)
        buf[:, t] = p.float()
        L += alive.to(torch.int64)
    keep = torch.arange(buf.shape[1], device=device)[None, :] < L[:, None]
    return buf[keep], L


def _lognormal_lengths(n, median, sigma, lo, hi, g, device):
    z = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    return torch.clamp(torch.round(torch.exp(math.log(median) + sigma * z)), lo, hi).to(torch.int64)


def _ellipsoid_inside(centre, semi, device):
    c = torch.tensor(centre, dtype=torch.float64, device=device)
    a = torch.tensor(semi, dtype=torch.float64, device=device)
    return lambda p: (((p - c) / a) ** 2).sum(-1) <= 1.0


def _assemble(name, vols: Volumes, chunks_pts, chunks_len, device, scale=1.0) -> Workload:
    points = torch.cat(chunks_pts) if chunks_pts else torch.zeros((0, 3), dtype=torch.float32, device=device)
    lens = torch.cat(chunks_len) if chunks_len else torch.zeros(0, dtype=torch.int64, device=device)
    offsets = torch.zeros(lens.shape[0] + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(lens, 0)
    return Workload(name, points.contiguous(), offsets, torch.from_numpy(vols.roi).to(device),
                    torch.from_numpy(vols.lab).to(device), vols.N, vols.M, scale)


def make_tiny64(seed: int = 1, S: int = 10_000, device="cpu") -> Workload:
    """64^3 case: S walks, lengths uniform in 20..200, 40% seeded uniformly in the ROI
    ellipsoid and 60% uniformly in the ball of radius 30; no mask stop."""
    vols = volumes_tiny64()
    pts, lens = [], []
    for c, a in enumerate(range(0, S, CHUNK)):
        n = min(CHUNK, S - a)
        g = _chunk_generator(seed, c, device)
        T = torch.randint(20, 201, (n,), generator=g, device=device)
        e = uniform_in_ellipsoid(n, (32.0, 32.0, 32.0), (10.0, 8.0, 7.0), g, device)
        b = uniform_in_ellipsoid(n, (32.0, 32.0, 32.0), (30.0, 30.0, 30.0), g, device)
        pick = torch.rand(n, generator=g, device=device, dtype=torch.float64) < 0.4
        seeds = torch.where(pick[:, None], e, b)
        p, L = random_walks(n, seeds, T, g, None)
        pts.append(p)
        lens.append(L)
    return _assemble("tiny64", vols, pts, lens, device)


def make_subject_walks(vols: Volumes, seed: int, S: int, median: float, lo: int, hi: int, device,
                       name: str, scale: float = 1.0) -> Workload:
    """S walks for an ellipsoidal subject: lognormal lengths (sigma 0.5) clipped to [lo,hi],
    40% seeded in one ROI ellipsoid (side drawn uniformly), 60% uniformly in the brain mask;
    a walk stops at its first step outside the mask."""
    inside = _ellipsoid_inside(vols.centre, vols.brain_semi, device)
    pts, lens = [], []
    (c0, a0), (c1, a1) = vols.roi_ellipsoids[0], vols.roi_ellipsoids[-1]
    for c, a in enumerate(range(0, S, CHUNK)):
        n = min(CHUNK, S - a)
        g = _chunk_generator(seed, c, device)
        T = _lognormal_lengths(n, median, 0.5, lo, hi, g, device)
        e0 = uniform_in_ellipsoid(n, c0, a0, g, device)
        e1 = uniform_in_ellipsoid(n, c1, a1, g, device)
        side = torch.rand(n, generator=g, device=device, dtype=torch.float64) < 0.5
        roi_seed = torch.where(side[:, None], e1, e0)
        brain_seed = uniform_in_ellipsoid(n, vols.centre, vols.brain_semi, g, device)
        pick = torch.rand(n, generator=g, device=device, dtype=torch.float64) < 0.4
        seeds = torch.where(pick[:, None], roi_seed, brain_seed)
        p, L = random_walks(n, seeds, T, g, inside)
        pts.append(p)
        lens.append(L)
    return _assemble(name, vols, pts, lens, device, scale)


def make_125mm(seed: int = 2, S: int = 1_000_000, device="cpu", vols: Optional[Volumes] = None) -> Workload:
    """1.25 mm-like subject: 145x174x145, N about 8k, M=70, lengths median 150 in [20,600]."""
    vols = vols or volumes_125mm(seed)
    return make_subject_walks(vols, seed, S, 150.0, 20, 600, device, "1.25mm")


def make_07mm(seed: int = 3, S: int = 5_000_000, device="cpu", vols: Optional[Volumes] = None) -> Workload:
    """0.7 mm-like subject: 260x311x260, N about 45.8k, M=180, lengths median 270 in [30,1000]."""
    vols = vols or volumes_07mm(seed)
    return make_subject_walks(vols, seed, S, 270.0, 30, 1000, device, "0.7mm")


def make_sr(seed: int = 5, S: int = 100_000, device="cpu", vols_lo: Optional[Volumes] = None,
            vols_hi: Optional[Volumes] = None) -> Workload:
    """Super-resolution job: walks drawn on the 1.25 mm subject, counted on the 0.7 mm volumes
    after scaling every coordinate by fl32(1.25/0.7)."""
    vols_lo = vols_lo or volumes_125mm(2)
    vols_hi = vols_hi or volumes_07mm(3)
    w = make_subject_walks(vols_lo, seed, S, 150.0, 20, 600, device, "sr")
    return Workload("sr", w.points, w.offsets, torch.from_numpy(vols_hi.roi).to(device),
                    torch.from_numpy(vols_hi.lab).to(device), vols_hi.N, vols_hi.M, SR_SCALE)


# ----------------------------------------------------------------------------------------------
# small adversarial inputs for parity and edge cases (numpy, host)
# ----------------------------------------------------------------------------------------------

def random_small(seed: int, dims=(12, 10, 9), S: int = 40, N: Optional[int] = None, M: int = 5,
                 roi_density: float = 0.3, lab_density: float = 0.3, max_len: int = 60,
                 specials: bool = True, bad_values: bool = False) -> Workload:
    """Tiny random case with revisits, out-of-grid points, empty and one-point streamlines,
    and (``specials``) NaN / inf / rounding-boundary coordinates.  ``bad_values`` also puts
    ROI / label values outside [0,N) / [0,M) into the volumes."""
    rng = np.random.default_rng([seed, 77])
    X, Y, Z = dims
    nvox = X * Y * Z
    roi = np.full(nvox, -1, dtype=np.int32)
    sel = rng.random(nvox) < roi_density
    n_roi = int(sel.sum())
    if N is None:
        N = max(1, n_roi)
        roi[sel] = np.arange(n_roi, dtype=np.int32) % N
    else:
        roi[sel] = rng.integers(0, N, size=n_roi, dtype=np.int32)   # several voxels may share a row
    lab = np.full(nvox, -1, dtype=np.int32)
    lsel = rng.random(nvox) < lab_density
    lab[lsel] = rng.integers(0, M, size=int(lsel.sum()), dtype=np.int32)
    if bad_values:
        k = rng.random(nvox)
        roi[k < 0.03] = N + rng.integers(0, 3)
        roi[(k >= 0.03) & (k < 0.05)] = -7
        lab[k > 0.97] = M + 1
    lens = rng.integers(0, max_len + 1, size=S)
    lens[rng.random(S) < 0.1] = 0
    lens[rng.random(S) < 0.1] = 1
    pts = []
    for T in lens:
        if T == 0:
            pts.append(np.zeros((0, 3), dtype=np.float32))
            continue
        p = rng.uniform(-1.5, 1.5, size=3) + rng.uniform(0, 1, size=3) * np.array(dims, dtype=np.float64)
        walk = [p.copy()]
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        for _ in range(int(T) - 1):
            if rng.random() < 0.15:          # U-turn: revisit voxels non-adjacently
                d = -d
            d = d + 0.6 * rng.normal(size=3)
            d /= np.linalg.norm(d)
            p = p + rng.choice([0.3, 0.5, 0.9, 1.7]) * d
            walk.append(p.copy())
        pts.append(np.asarray(walk, dtype=np.float32).reshape(-1, 3))
    P = np.concatenate(pts) if pts else np.zeros((0, 3), dtype=np.float32)
    if specials and P.shape[0]:
        k = rng.random(P.shape)
        P[k < 0.01] = np.nan
        P[(k >= 0.01) & (k < 0.015)] = np.inf
        P[(k >= 0.015) & (k < 0.02)] = -np.inf
        P[(k >= 0.02) & (k < 0.04)] = np.float32(0.49999997)
        P[(k >= 0.04) & (k < 0.06)] = np.float32(-0.5)
        edge = (k >= 0.06) & (k < 0.08)
        P[edge] = (np.broadcast_to(np.array(dims, dtype=np.float32), P.shape)[edge] - np.float32(0.5))
    off = np.zeros(S + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    return Workload(f"small{seed}", torch.from_numpy(P.astype(np.float32)), torch.from_numpy(off),
                    torch.from_numpy(roi.reshape(Z, Y, X)), torch.from_numpy(lab.reshape(Z, Y, X)),
                    int(N), int(M))


# ----------------------------------------------------------------------------------------------
# batched form: subjects of uneven grid size, N, M and streamline count
# ----------------------------------------------------------------------------------------------

def volumes_batch_subject(k: int, seed: int = 4) -> Volumes:
    """Subject k of the batched workload (seeded from seed*1000 + k): grid dims drawn per axis between
    the 64^3 and the 1.25 mm sizes; brain ellipsoid proportional to the grid; a bilateral ROI of the
    1.25 mm shape scaled to a target N drawn in [5k, 45k] (at most 30% of the mask); M drawn from
    {70, 180, 360} labels on a 3-voxel shell."""
    rng = np.random.default_rng([seed * 1000 + k, 1])
    dims = (int(rng.integers(64, 146)), int(rng.integers(64, 175)), int(rng.integers(64, 146)))
    X, Y, Z = dims
    centre = ((X - 1) / 2.0, (Y - 1) / 2.0, (Z - 1) / 2.0)
    brain = (X * 56.0 / 145.0, Y * 68.0 / 174.0, Z * 52.0 / 145.0)
    ratio = tuple(d / float(c) for d, c in zip(dims, CFG2_DIMS))
    n_target = float(rng.uniform(5000, 45000))
    mask_vol = 4.0 / 3.0 * math.pi * brain[0] * brain[1] * brain[2]
    base_vol = 2 * 4.0 / 3.0 * math.pi * CFG2_ROI_SEMI[0] * CFG2_ROI_SEMI[1] * CFG2_ROI_SEMI[2]
    f = min(n_target, 0.3 * mask_vol) / base_vol
    semi = tuple(a * f ** (1.0 / 3.0) for a in CFG2_ROI_SEMI)
    centres = [tuple(centre[i] + (rc[i] - CFG2_CENTRE[i]) * ratio[i] for i in range(3)) for rc in CFG2_ROI_CENTRES]
    M = int(rng.choice([70, 180, 360]))
    return volumes_subject(dims, centre, brain, semi, centres, M, 3.0, rng)


def make_batch_subject(k: int, seed: int = 4, device="cpu", S: Optional[int] = None,
                       vols: Optional[Volumes] = None) -> Workload:
    """Streamlines of batched subject k: S drawn in [100k, 2M] (unless given), lengths as in the
    1.25 mm recipe, walks stopping at the brain mask."""
    vols = vols or volumes_batch_subject(k, seed)
    if S is None:
        S = int(np.random.default_rng([seed * 1000 + k, 2]).integers(100_000, 2_000_001))
    return make_subject_walks(vols, seed * 1000 + k, S, 150.0, 20, 600, device, f"batch{k}")

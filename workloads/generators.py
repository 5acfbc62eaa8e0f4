"""Seeded synthetic planar straight-line graphs (PSLGs).

The paper refines contour maps and synthetic sets that are not available here
(Section 7.1, Table 1), so these generators stand in for them.  Every input is
drawn from ``numpy.random.Generator(PCG64(seed))``; ``manifest_hash`` gives a
SHA-256 over the arrays so a drift in the numpy streams is detected by the
tests.

Conventions shared by all generators:

* vertices 0..3 are the unit-square corners (0,0), (1,0), (1,1), (0,1);
* segments 0..3 are the square's sides (0,1), (1,2), (2,3), (3,0), so the
  convex hull is covered by constraint segments (the refinement domain is the
  square, Section 4 problem statement);
* ``ratio_bound_sq`` is the squared radius-edge bound B^2 passed as an FP64
  literal (B = sqrt(2) -> 2.0).

Rejection rules for constraint segments (same for every config): a candidate
segment is rejected if it crosses or touches an accepted segment away from a
shared endpoint, if it passes within ``1e-6`` of any point other than its own
endpoints, or if it makes an angle below 60 degrees with an accepted segment at
a shared endpoint.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

PROX = 1e-6          # minimum point-to-segment clearance
MIN_ANGLE_DEG = 60.0  # minimum angle between segments at a shared endpoint
COS_MIN = math.cos(math.radians(MIN_ANGLE_DEG))

CORNERS = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]], dtype=np.float64)
BOUNDARY = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], dtype=np.int32)


@dataclass
class PSLG:
    name: str
    xy: np.ndarray              # (n, 2) float64
    seg: np.ndarray             # (m, 2) int32
    ratio_bound_sq: float = 2.0
    meta: dict = field(default_factory=dict)

    @property
    def n_vertices(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_segments(self) -> int:
        return int(self.seg.shape[0])


def manifest_hash(p: PSLG) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(p.xy, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(p.seg, dtype="<i4").tobytes())
    h.update(np.float64(p.ratio_bound_sq).tobytes())
    return h.hexdigest()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _inside_mask(pts: np.ndarray) -> np.ndarray:
    return np.all((pts >= PROX) & (pts <= 1.0 - PROX), axis=1)


def _uniform_inside(rng, n: int) -> np.ndarray:
    out = rng.random((n, 2))
    bad = ~_inside_mask(out)
    while bad.any():
        out[bad] = rng.random((int(bad.sum()), 2))
        bad = ~_inside_mask(out)
    return out


def _dedupe(rng, pts: np.ndarray, redraw) -> np.ndarray:
    """Redraw exact duplicate points (vanishingly rare) with ``redraw(k)``."""
    while True:
        _, idx, counts = np.unique(pts, axis=0, return_index=True, return_counts=True)
        if (counts == 1).all():
            return pts
        keep = np.zeros(len(pts), dtype=bool)
        keep[idx] = True
        dup = ~keep
        pts[dup] = redraw(int(dup.sum()))


# ---------------------------------------------------------------------------
# Segment acceptance with a uniform grid (points and accepted segments)
# ---------------------------------------------------------------------------

class _SegmentSet:
    def __init__(self, xy: np.ndarray, cell: float):
        self.xy = xy
        self.cell = cell
        self.ng = max(1, int(math.ceil(1.0 / cell)))
        g = np.clip((xy / cell).astype(np.int64), 0, self.ng - 1)
        key = g[:, 0] * self.ng + g[:, 1]
        order = np.argsort(key, kind="stable")
        self.pt_order = order
        sk = key[order]
        self.pt_start = np.searchsorted(sk, np.arange(self.ng * self.ng), side="left")
        self.pt_end = np.searchsorted(sk, np.arange(self.ng * self.ng), side="right")
        self.seg_cells: dict[int, list[int]] = {}
        self.segs: list[tuple[int, int]] = []
        self.inc: dict[int, list[int]] = {}
        self.keys: set[tuple[int, int]] = set()

    def _cells(self, a: np.ndarray, b: np.ndarray, pad: float):
        lo = np.minimum(a, b) - pad
        hi = np.maximum(a, b) + pad
        i0, j0 = (np.clip((lo / self.cell).astype(np.int64), 0, self.ng - 1))
        i1, j1 = (np.clip((hi / self.cell).astype(np.int64), 0, self.ng - 1))
        for i in range(i0, i1 + 1):
            for j in range(j0, j1 + 1):
                yield i * self.ng + j

    def try_add(self, ia: int, ib: int) -> bool:
        if ia == ib:
            return False
        key = (min(ia, ib), max(ia, ib))
        if key in self.keys:
            return False
        xy = self.xy
        a, b = xy[ia], xy[ib]
        d = b - a
        L2 = float(d @ d)
        if L2 <= 0.0:
            return False
        cells = list(self._cells(a, b, PROX))
        # clearance to all other points
        idx = [self.pt_order[self.pt_start[c]:self.pt_end[c]] for c in cells]
        idx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
        idx = idx[(idx != ia) & (idx != ib)]
        if idx.size:
            q = xy[idx] - a
            t = np.clip((q @ d) / L2, 0.0, 1.0)
            r = q - t[:, None] * d
            if np.min(np.einsum("ij,ij->i", r, r)) < PROX * PROX:
                return False
        # angle at shared endpoints
        for (iv, other) in ((ia, ib), (ib, ia)):
            for s in self.inc.get(iv, ()):
                u, v = self.segs[s]
                w = v if u == iv else u
                e1 = xy[other] - xy[iv]
                e2 = xy[w] - xy[iv]
                c = float(e1 @ e2) / math.sqrt(float(e1 @ e1) * float(e2 @ e2))
                if c > COS_MIN:
                    return False
        # crossing / touching with accepted segments
        seen = set()
        for c in cells:
            for s in self.seg_cells.get(c, ()):
                if s in seen:
                    continue
                seen.add(s)
                u, v = self.segs[s]
                if u in (ia, ib) or v in (ia, ib):
                    continue  # shared endpoint handled by the angle rule
                if _segments_meet(a, b, xy[u], xy[v]):
                    return False
        sid = len(self.segs)
        self.segs.append((ia, ib))
        self.keys.add(key)
        self.inc.setdefault(ia, []).append(sid)
        self.inc.setdefault(ib, []).append(sid)
        for c in cells:
            self.seg_cells.setdefault(c, []).append(sid)
        return True


def _orient(a, b, c) -> float:
    return (a[0] - c[0]) * (b[1] - c[1]) - (a[1] - c[1]) * (b[0] - c[0])


def _segments_meet(a, b, c, d) -> bool:
    """Conservative crossing test: True when the segments cross or nearly touch.

    Endpoints are at least ``PROX`` away from the other segment (checked
    first), so the orientation magnitudes are far above FP64 rounding.
    """
    d1 = _orient(a, b, c)
    d2 = _orient(a, b, d)
    d3 = _orient(c, d, a)
    d4 = _orient(c, d, b)
    return (d1 * d2 <= 0.0) and (d3 * d4 <= 0.0)


def _assemble(name, interior: np.ndarray, segs: list[tuple[int, int]], offset: int,
              bsq: float, meta: dict) -> PSLG:
    xy = np.concatenate([CORNERS, interior]).astype(np.float64)
    s = np.asarray(segs, dtype=np.int64).reshape(-1, 2) + offset
    seg = np.concatenate([BOUNDARY, s.astype(np.int32)]).astype(np.int32)
    return PSLG(name=name, xy=np.ascontiguousarray(xy), seg=np.ascontiguousarray(seg),
                ratio_bound_sq=float(bsq), meta=meta)


# ---------------------------------------------------------------------------
# Configs
# ---------------------------------------------------------------------------

def bare_square() -> PSLG:
    """Four corners and the four sides: the smallest valid domain."""
    return PSLG("bare_square", CORNERS.copy(), BOUNDARY.copy(), 2.0, {})


def near_edge_point(delta: float = 1e-3) -> PSLG:
    """The square plus one interior point at distance ``delta`` above the bottom side."""
    xy = np.concatenate([CORNERS, np.array([[0.5, delta]])])
    return PSLG("near_edge_point", xy, BOUNDARY.copy(), 2.0, {"delta": delta})


def random_small(seed: int, n_points: int, n_segments: int, bsq: float = 2.0,
                 pairing: str = "uniform", max_attempts: int = 200_000) -> PSLG:
    """Config-0 style PSLG of any size (uniform points, rejected random segments)."""
    rng = _rng(seed)
    pts = _uniform_inside(rng, n_points)
    pts = _dedupe(rng, pts, lambda k: _uniform_inside(rng, k))
    cell = 1.0 / 32 if pairing == "uniform" else max(1e-3, 2.0 / math.sqrt(max(n_points, 1)))
    ss = _SegmentSet(pts, cell)
    if pairing == "knn" and n_points > 1:
        nbr = _knn(pts, 16)
    attempts = 0
    while len(ss.segs) < n_segments:
        attempts += 1
        if attempts > max_attempts:
            raise RuntimeError(f"segment rejection exceeded {max_attempts} attempts")
        if pairing == "uniform":
            ia, ib = (int(v) for v in rng.integers(0, n_points, size=2))
        else:
            ia = int(rng.integers(0, n_points))
            ib = int(nbr[ia, int(rng.integers(0, nbr.shape[1]))])
        ss.try_add(ia, ib)
    return _assemble(f"random_small_s{seed}_n{n_points}_m{n_segments}", pts, ss.segs, 4, bsq,
                     {"seed": seed, "attempts": attempts, "pairing": pairing})


def config0(seed: int = 0) -> PSLG:
    """1,000 uniform points + 50 uniformly paired segments + square; B = sqrt(2)."""
    p = random_small(seed, 1000, 50, 2.0, pairing="uniform")
    p.name = "c0_1k_uniform"
    return p


def _knn(pts: np.ndarray, k: int) -> np.ndarray:
    from scipy.spatial import cKDTree
    tree = cKDTree(pts)
    _, idx = tree.query(pts, k=k + 1)
    return idx[:, 1:]


def _c1_points(rng, n: int) -> np.ndarray:
    n_u = n - 2 * (n // 3)
    n_c = n // 3
    n_e = n // 3
    uni = _uniform_inside(rng, n_u)
    centres = rng.random((64, 2))
    which = rng.integers(0, 64, size=n_c)
    clu = centres[which] + rng.normal(0.0, 0.01, size=(n_c, 2))
    bad = ~_inside_mask(clu)
    while bad.any():
        clu[bad] = centres[which[bad]] + rng.normal(0.0, 0.01, size=(int(bad.sum()), 2))
        bad = ~_inside_mask(clu)
    t = rng.random(n_e) * (2.0 * math.pi)
    ell = np.stack([0.5 + 0.45 * np.cos(t), 0.5 + 0.3 * np.sin(t)], axis=1)
    ell = ell + rng.normal(0.0, 1e-4, size=(n_e, 2))
    pts = np.concatenate([uni, clu, ell])
    return _dedupe(rng, pts, lambda k: _uniform_inside(rng, k))


def scaled_config1(n: int, n_segments: int, seed: int = 1, bsq: float = 2.0) -> PSLG:
    """Config-1 generator at any size: uniform / 64 Gaussian clusters / jittered ellipse
    thirds, plus k-nearest-neighbour paired segments (one of the 16 nearest, uniformly)."""
    rng = _rng(seed)
    pts = _c1_points(rng, n)
    nbr = _knn(pts, 16)
    cell = max(2e-4, 4.0 / math.sqrt(n))
    ss = _SegmentSet(pts, cell)
    attempts = 0
    limit = 20 * n_segments + 1000
    while len(ss.segs) < n_segments:
        batch = rng.integers(0, n, size=4096)
        pick = rng.integers(0, 16, size=4096)
        for ia, j in zip(batch.tolist(), pick.tolist()):
            attempts += 1
            if ss.try_add(ia, int(nbr[ia, j])) and len(ss.segs) >= n_segments:
                break
        if attempts > limit:
            raise RuntimeError("segment rejection exceeded its attempt budget")
    return _assemble(f"c1_like_n{n}_m{n_segments}_s{seed}", pts, ss.segs, 4, bsq,
                     {"seed": seed, "attempts": attempts})


def config1(seed: int = 1) -> PSLG:
    """1,000,000 points (uniform / clusters / ellipse) + 50,000 kNN segments + square."""
    p = scaled_config1(1_000_000, 50_000, seed)
    p.name = "c1_1M_mixed"
    return p


def scaled_config2(n_circles: int, per_circle: int, n_free: int, seed: int = 2,
                   r_lo: float = 0.01, r_hi: float = 0.49, gap: float = 1e-4,
                   bsq: float = 2.0) -> PSLG:
    """Concentric closed polygons about (0.5, 0.5) plus uniform free points."""
    rng = _rng(seed)
    radii: list[float] = []
    while len(radii) < n_circles:
        r = float(rng.uniform(r_lo, r_hi))
        if all(abs(r - q) >= gap for q in radii):
            radii.append(r)
    radii.sort()
    radii_a = np.asarray(radii)
    phase = rng.random(n_circles) * (2.0 * math.pi)
    j = np.arange(per_circle)
    circ = []
    segs = []
    step = 2.0 * math.pi / per_circle
    for ci, (r, ph) in enumerate(zip(radii, phase)):
        ang = j * step + ph
        circ.append(np.stack([0.5 + r * np.cos(ang), 0.5 + r * np.sin(ang)], axis=1))
        base = ci * per_circle
        segs.append(np.stack([base + j, base + (j + 1) % per_circle], axis=1))
    circ_xy = np.concatenate(circ) if circ else np.zeros((0, 2))
    seg_arr = np.concatenate(segs) if segs else np.zeros((0, 2), np.int64)

    def clearance_ok(p: np.ndarray) -> np.ndarray:
        dx = p[:, 0] - 0.5
        dy = p[:, 1] - 0.5
        rho = np.hypot(dx, dy)
        ok = _inside_mask(p)
        if n_circles == 0:
            return ok
        pos = np.searchsorted(radii_a, rho)
        theta = np.mod(np.arctan2(dy, dx), 2.0 * math.pi)
        for off in (-1, 0):
            ci = np.clip(pos + off, 0, n_circles - 1)
            near = np.abs(rho - radii_a[ci]) < 1e-4
            if not near.any():
                continue
            sel = np.nonzero(near)[0]
            for s in sel.tolist():
                c = int(ci[s])
                k = int(np.floor(np.mod(theta[s] - phase[c], 2.0 * math.pi) / step))
                for kk in (k - 1, k, k + 1):
                    a = circ_xy[c * per_circle + (kk % per_circle)]
                    b = circ_xy[c * per_circle + ((kk + 1) % per_circle)]
                    d = b - a
                    q = p[s] - a
                    t = min(1.0, max(0.0, float(q @ d) / float(d @ d)))
                    rr = q - t * d
                    if float(rr @ rr) < PROX * PROX:
                        ok[s] = False
        return ok

    free = rng.random((n_free, 2))
    ok = clearance_ok(free)
    while not ok.all():
        bad = ~ok
        free[bad] = rng.random((int(bad.sum()), 2))
        ok = clearance_ok(free)
    interior = np.concatenate([circ_xy, free])
    interior = _dedupe(rng, interior, lambda k: rng.random((k, 2)))
    return _assemble(f"c2_like_c{n_circles}x{per_circle}_f{n_free}_s{seed}", interior,
                     [tuple(s) for s in seg_arr.tolist()], 4, bsq,
                     {"seed": seed, "radii": radii_a})


def config2(seed: int = 2) -> PSLG:
    """512 concentric 1000-gons (512,000 segments) + 100,000 free points + square."""
    p = scaled_config2(512, 1000, 100_000, seed)
    p.name = "c2_512_circles"
    return p


# ---- batched form (4,096 independent PSLGs) ---------------------------------
BATCH_BOUNDS_SQ = (2.0, 2.56, 4.0)  # B = sqrt(2), 1.6, 2.0, passed squared as FP64 literals


def batch_plan(count: int = 4096, seed: int = 3, n_min: int = 100, n_max: int = 50_000):
    """Sizes (log-uniform in [n_min, n_max]), bounds and per-instance seeds."""
    rng = _rng(seed)
    n = np.floor(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=count))).astype(np.int64)
    bsq = rng.choice(np.array(BATCH_BOUNDS_SQ), size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return n, bsq, seeds


def batch_instance(n: int, bsq: float, seed: int) -> PSLG:
    """One instance: config-0 style uniform points, k-nearest-neighbour
    segments (5% of the vertices), unit square."""
    m = max(1, int(round(0.05 * n)))
    p = random_small(int(seed), int(n), m, float(bsq), pairing="knn")
    p.name = f"c3_s{int(seed)}_n{int(n)}"
    return p


def _batch_instance_args(args):
    return batch_instance(*args)


def batch_config3(count: int = 4096, seed: int = 3, n_min: int = 100, n_max: int = 50_000,
                  workers: int = 1) -> list[PSLG]:
    """The batched workload: count instances of batch_instance (generated in
    parallel when workers > 1; each instance depends only on its own seed)."""
    n, bsq, seeds = batch_plan(count, seed, n_min, n_max)
    args = list(zip(n.tolist(), bsq.tolist(), seeds.tolist()))
    if workers > 1 and count > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            return pool.map(_batch_instance_args, args, chunksize=8)
    return [batch_instance(*a) for a in args]


# ---- serving form (a stream of jobs of mixed sizes) --------------------------
def serving_plan(count: int, seed: int = 4, n_min: int = 1_000, n_max: int = 200_000):
    """Sizes (log-uniform), bounds and per-job seeds of a job stream."""
    rng = _rng(seed)
    n = np.floor(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=count))).astype(np.int64)
    bsq = rng.choice(np.array(BATCH_BOUNDS_SQ), size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return n, bsq, seeds


def serving_job(n: int, bsq: float, seed: int) -> PSLG:
    """One job: the 1M-point generator scaled to n points, segments 5% of them."""
    p = scaled_config1(int(n), max(1, int(round(0.05 * n))), seed=int(seed), bsq=float(bsq))
    p.name = f"c4_s{int(seed)}_n{int(n)}"
    return p


def _serving_job_args(args):
    return serving_job(*args)


def serving_jobs(count: int, seed: int = 4, n_min: int = 1_000, n_max: int = 200_000,
                 workers: int = 1) -> list[PSLG]:
    n, bsq, seeds = serving_plan(count, seed, n_min, n_max)
    args = list(zip(n.tolist(), bsq.tolist(), seeds.tolist()))
    if workers > 1 and count > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            return pool.map(_serving_job_args, args, chunksize=2)
    return [serving_job(*a) for a in args]


def spokes(deg: float, n_spokes: int = 4, n_free: int = 200, seed: int = 3, length: float = 0.45) -> PSLG:
    """Small input angles: the square, n_free uniform points and n_spokes segments
    of the given length from one input vertex at (0.31, 0.37), deg degrees apart
    (the first at 10 degrees).  B = sqrt(2)."""
    import math
    rng = _rng(seed)
    pts = CORNERS.tolist() + [[0.31, 0.37]]
    seg = BOUNDARY.tolist()
    for i in range(n_spokes):
        a = math.radians(10.0 + deg * i)
        pts.append([0.31 + length * math.cos(a), 0.37 + length * math.sin(a)])
        seg.append([4, len(pts) - 1])
    pts += rng.uniform(0.02, 0.98, size=(n_free, 2)).tolist()
    return PSLG(f"spokes_{deg:g}deg", np.array(pts, dtype=np.float64), np.array(seg, dtype=np.int32), 2.0,
                {"deg": deg, "n_spokes": n_spokes, "n_free": n_free, "seed": seed})

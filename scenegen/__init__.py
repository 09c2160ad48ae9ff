"""Seeded synthetic reconstructions (inputs only).

This module produces the *inputs* of the camera-covariance computation:
cameras, points and the observation index set S (paper, Sec. 4, "Problem
formulation").  It holds none of the method's arithmetic: no projection
model, no Jacobian, no normal equations.  Camera orientations are built as
look-at frames and converted to angle-axis with SciPy; visibility is a
field-of-view test on those frames (a point is seen when it lies in front of
the camera within the 640 x 480 frame's viewing cone), with no focal length,
distortion or derivative involved.

Both the CPU oracle (through the tests) and the GPU library (through the
Python binding) consume the same ``Scene`` objects, so neither side generates
its own inputs.

Camera parameter layout, one row of 9 float64 per camera, in the order the
paper uses for P_i = {r_i, C_i, c_i, k_i} (Sec. 5.1) extended to two radial
coefficients:

    r0 r1 r2   angle-axis of the world-to-camera rotation R(r)
    C0 C1 C2   camera centre in world coordinates
    f          focal length in pixels
    k1 k2      radial distortion coefficients

Recipes (all distributions are seeded with numpy's PCG64 ``default_rng``):

* ``tiny_circle``   10 cameras on a circle of radius 10 in the z=0 plane looking
  at the origin (up = +z); 200 points uniform in a ball of radius 3; every
  point is seen by 3..6 distinct random cameras; f = 1000*U[0.95,1.05];
  k1, k2 ~ N(0, 0.1^2).  Z is 90 x 90.
* ``spiral_slab``   n cameras (default 500) on an Archimedean spiral of three
  turns at height 8 above the slab [-10,10]^2 x [-2.5,2.5] (radius 1.5 -> 7.4,
  per-axis jitter N(0, 0.2^2)), nadir-looking with a N(0, (2 deg)^2) tilt;
  m points (default 50 000) in the slab, each drawn on the viewing ray of a
  random pixel of a random camera at a height uniform in the slab and kept
  when at least two cameras see it; track length t = 1 + Geometric(p) (mean
  6 for p = 0.2, minimum 2, capped at 30 and at the number of cameras that
  see the point), the track's cameras drawn at random from the 2t nearest
  cameras that see the point.  Z is 9n x 9n (4500 x 4500 by default).
* ``clustered``     10 clusters of 300 cameras on a ring of radius 40 and
  500 000 points, Zipf(1.5) track lengths on [2, 30], 2 % of the tracks
  spanning two adjacent clusters and 5 % of the points placed so far away
  that their triangulation angle is about 1e-4 rad (near-zero baseline).
* ``batch_scenes``  256 independent spiral scenes with camera counts
  log-uniform in [20, 400], 100 points per camera and mean track length 5;
  scene s is a stretch of 3 n_s / 500 turns of the spiral above, so that the
  camera spacing and the overlap of neighbouring views are those of the
  500-camera scene.

The observed image coordinates (and their 1 px noise) are not generated: a
first-order covariance does not depend on the residuals (Sec. 4, the normal
equations), so the library never reads them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

PRINCIPAL_POINT = (320.0, 240.0)  # 640 x 480 image, fixed, not a parameter


@dataclasses.dataclass
class Scene:
    """A reconstruction theta = {P, X} with its index set S."""

    cams: np.ndarray       # (n, 9) float64
    pts: np.ndarray        # (m, 3) float64
    obs_cam: np.ndarray    # (t,) int32
    obs_pt: np.ndarray     # (t,) int32
    obs_info: np.ndarray | None = None  # (t, 3) float64: a, b, c of [[a, b], [b, c]]
    name: str = ""
    seed: int = 0

    @property
    def n_cams(self) -> int:
        return int(self.cams.shape[0])

    @property
    def n_pts(self) -> int:
        return int(self.pts.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_cam.shape[0])

    def subset_points(self, keep: np.ndarray) -> "Scene":
        """Same cameras, only the points whose mask entry is true."""
        keep = np.asarray(keep, bool)
        new_index = -np.ones(self.n_pts, np.int64)
        new_index[keep] = np.arange(int(keep.sum()))
        sel = keep[self.obs_pt]
        info = None if self.obs_info is None else self.obs_info[sel].copy()
        return Scene(self.cams.copy(), self.pts[keep].copy(),
                     self.obs_cam[sel].astype(np.int32),
                     new_index[self.obs_pt[sel]].astype(np.int32), info,
                     self.name + "-sub", self.seed)


# ----------------------------------------------------------------------------
# helpers (geometry of the synthetic rig only)
# ----------------------------------------------------------------------------

def _look_at_rotvec(centres: np.ndarray, forward: np.ndarray, up: np.ndarray) -> np.ndarray:
    """Angle-axis of world-to-camera rotations whose third row is ``forward``."""
    z = forward / np.linalg.norm(forward, axis=1, keepdims=True)
    x = np.cross(z, up)
    bad = np.linalg.norm(x, axis=1) < 1e-9
    if bad.any():
        x[bad] = np.cross(z[bad], np.array([1.0, 0.0, 0.0]))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    rows = np.stack([x, y, z], axis=1)  # rows are the camera axes in world coords
    return Rotation.from_matrix(rows).as_rotvec()


def _intrinsics(rng: np.random.Generator, n: int) -> np.ndarray:
    f = 1000.0 * rng.uniform(0.95, 1.05, n)
    k = rng.normal(0.0, 0.1, (n, 2))
    return np.column_stack([f, k])


def _check_connected(n: int, obs_cam: np.ndarray, obs_pt: np.ndarray) -> None:
    """Cameras and points must form one connected component (nullity 7)."""
    m = int(obs_pt.max()) + 1
    g = coo_matrix((np.ones(obs_cam.size), (obs_cam, n + obs_pt)), shape=(n + m, n + m))
    ncomp, _ = connected_components(g, directed=False)
    if ncomp != 1:
        raise RuntimeError(f"generated scene is not connected ({ncomp} components)")


def _finish(rng, cams, pts, tracks, name, seed, with_info) -> Scene:
    obs_cam = np.concatenate(tracks).astype(np.int32)
    obs_pt = np.repeat(np.arange(len(tracks)), [len(t) for t in tracks]).astype(np.int32)
    perm = rng.permutation(obs_cam.size)  # observation order is arbitrary at the boundary
    obs_cam, obs_pt = obs_cam[perm], obs_pt[perm]
    _check_connected(cams.shape[0], obs_cam, obs_pt)
    info = None
    if with_info:
        info = random_information(rng, obs_cam.size)
    return Scene(np.ascontiguousarray(cams, np.float64), np.ascontiguousarray(pts, np.float64),
                 obs_cam, obs_pt, info, name, seed)


def random_information(rng: np.random.Generator, t: int) -> np.ndarray:
    """Per-observation 2x2 information matrices Sigma_u^-1 (eigenvalues of
    Sigma_u in [0.5, 2] px^2, random orientation), stored as (a, b, c)."""
    ang = rng.uniform(0, np.pi, t)
    ev = rng.uniform(0.5, 2.0, (t, 2))
    c, s = np.cos(ang), np.sin(ang)
    # Sigma_u^-1 = R diag(1/ev) R^T
    l0, l1 = 1.0 / ev[:, 0], 1.0 / ev[:, 1]
    a = c * c * l0 + s * s * l1
    b = c * s * (l0 - l1)
    d = s * s * l0 + c * c * l1
    return np.column_stack([a, b, d])


# ----------------------------------------------------------------------------
# recipes
# ----------------------------------------------------------------------------

def tiny_circle(seed: int = 0, n: int = 10, m: int = 200, radius: float = 10.0,
                ball: float = 3.0, track=(3, 6), with_info: bool = False) -> Scene:
    """10 cameras on a circle looking at the origin, 200 points in a ball."""
    rng = np.random.default_rng(seed)
    ang = 2 * np.pi * np.arange(n) / n
    centres = radius * np.column_stack([np.cos(ang), np.sin(ang), np.zeros(n)])
    rot = _look_at_rotvec(centres, -centres, np.tile([0.0, 0.0, 1.0], (n, 1)))
    cams = np.column_stack([rot, centres, _intrinsics(rng, n)])
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = d * (ball * rng.uniform(0, 1, m) ** (1 / 3))[:, None]
    tracks = [rng.choice(n, size=min(n, int(rng.integers(track[0], track[1] + 1))), replace=False)
              for _ in range(m)]
    return _finish(rng, cams, pts, tracks, "tiny_circle", seed, with_info)


def _look_at_axes(forward: np.ndarray, up: np.ndarray) -> np.ndarray:
    """Rows x, y, z of look-at camera frames (z = viewing direction)."""
    z = forward / np.linalg.norm(forward, axis=1, keepdims=True)
    x = np.cross(z, up)
    bad = np.linalg.norm(x, axis=1) < 1e-9
    if bad.any():
        x[bad] = np.cross(z[bad], np.array([1.0, 0.0, 0.0]))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return np.stack([x, np.cross(z, x), z], axis=1)


def _spiral_cameras(rng, n, scale, turns=3.0):
    # Archimedean spiral r = scale*(0.15 + 0.59 theta/(2 pi turns)), cameras at
    # equal arc-length spacing along it; the outer end (0.74 scale) keeps every
    # camera's ground footprint (half-width 0.26 scale) inside the slab
    fine = np.linspace(0.0, 2 * np.pi * turns, 20001)
    r_f = scale * (0.15 + 0.59 * fine / (2 * np.pi * turns))
    ds = np.hypot(np.diff(r_f), 0.5 * (r_f[1:] + r_f[:-1]) * np.diff(fine))
    arc = np.concatenate([[0.0], np.cumsum(ds)])
    theta = np.interp(np.linspace(0.0, arc[-1], n), arc, fine)
    rad = scale * (0.15 + 0.59 * theta / (2 * np.pi * turns))
    centres = np.column_stack([rad * np.cos(theta), rad * np.sin(theta),
                               np.full(n, 0.8 * scale)])
    centres += rng.normal(0.0, 0.02 * scale, (n, 3))
    tilt = Rotation.from_rotvec(rng.normal(0.0, np.deg2rad(2.0), (n, 3)))
    forward = tilt.apply(np.array([0.0, 0.0, -1.0]))
    up = np.column_stack([np.cos(theta), np.sin(theta), np.zeros(n)])  # radial direction
    axes = _look_at_axes(forward, up)
    rot = Rotation.from_matrix(axes).as_rotvec()
    return np.column_stack([rot, centres, _intrinsics(rng, n)]), axes


# Field of view used for visibility: a point is seen by a camera when it lies
# in front of it inside the 640 x 480 frame of a 1000 px focal length
# (half-angle tangents 0.32 and 0.24, kept slightly inside the frame).
_FOV_TAN = (0.30, 0.22)


def _in_view(axes, centres, pts, cand, chunk=4096):
    """(m, K) mask: candidate camera cand[j, k] sees point j."""
    cen = [np.ascontiguousarray(centres[:, c]) for c in range(3)]
    ax = [[np.ascontiguousarray(axes[:, i, c]) for c in range(3)] for i in range(3)]
    out = np.empty(cand.shape, dtype=bool)
    for j0 in range(0, cand.shape[0], chunk):
        cj = cand[j0:j0 + chunk]
        d = [pts[j0:j0 + chunk, None, c] - cen[c][cj] for c in range(3)]   # (chunk, K) each
        xc = [sum(ax[i][c][cj] * d[c] for c in range(3)) for i in range(3)]
        z = xc[2]
        out[j0:j0 + chunk] = ((z > 0) & (np.abs(xc[0]) <= _FOV_TAN[0] * z)
                              & (np.abs(xc[1]) <= _FOV_TAN[1] * z))
    return out


def spiral_slab(seed: int = 0, n: int = 500, m: int = 50_000, p_geom: float = 0.2,
                scale: float = 10.0, with_info: bool = False, max_track: int = 30,
                turns: float = 3.0) -> Scene:
    """Cameras on a noisy spiral above a slab of points (nadir views).

    With the default ``scale`` of 10 the spiral radius runs 1.5 -> 7.4 at
    height 8 and the slab is [-10,10]^2 x [-2.5,2.5].  Every point lies in the view of
    at least two cameras; its track is drawn among the cameras that see it.
    """
    rng = np.random.default_rng(seed)
    cams, axes = _spiral_cameras(rng, n, scale, turns)
    centres = cams[:, 3:6]
    tree = cKDTree(centres)
    K = int(min(n, 2 * max_track + 20))
    pts_l, cand_l, vis_l = [], [], []
    have = 0
    rounds = 0
    while have < m:
        rounds += 1
        if rounds > 200:
            raise RuntimeError("spiral_slab: too few points are seen by two cameras "
                               f"({have} of {m}); use more cameras")
        b = int(1.3 * (m - have)) + 64
        # a ray through a random pixel of a random camera, cut at a random
        # height of the slab
        a = rng.integers(0, n, b)
        ray = np.column_stack([rng.uniform(-_FOV_TAN[0], _FOV_TAN[0], b),
                               rng.uniform(-_FOV_TAN[1], _FOV_TAN[1], b), np.ones(b)])
        ray = (axes[a] * ray[:, :, None]).sum(axis=1)          # R^T ray: to world coordinates
        zt = rng.uniform(-0.25 * scale, 0.25 * scale, b)
        p = centres[a] + ray * ((zt - centres[a, 2]) / ray[:, 2])[:, None]
        ok = (np.abs(p[:, 0]) <= scale) & (np.abs(p[:, 1]) <= scale)
        p = p[ok]
        _, cand = tree.query(p, k=K, workers=-1)
        cand = np.atleast_2d(cand).reshape(p.shape[0], K)
        vis = _in_view(axes, centres, p, cand)
        keep = vis.sum(axis=1) >= 2
        pts_l.append(p[keep])
        cand_l.append(cand[keep])
        vis_l.append(vis[keep])
        have += int(keep.sum())
    pts = np.concatenate(pts_l)[:m]
    cand = np.concatenate(cand_l)[:m]
    vis = np.concatenate(vis_l)[:m]
    nvis = vis.sum(axis=1)
    t = np.minimum(np.minimum(1 + rng.geometric(p_geom, m), max_track), nvis)
    # t_j distinct cameras uniformly among the 2 t_j nearest cameras that see
    # the point: random keys, every other candidate masked out, the t_j
    # smallest keys kept
    rank = np.cumsum(vis, axis=1) - 1                          # rank among the visible ones
    allowed = vis & (rank < 2 * t[:, None])
    keys = rng.random((m, K))
    keys[~allowed] = np.inf
    tmax = int(t.max())
    part = np.argpartition(keys, tmax - 1, axis=1)[:, :tmax]    # the tmax smallest, unordered
    part = np.take_along_axis(part, np.argsort(np.take_along_axis(keys, part, axis=1), axis=1), axis=1)
    picked = np.take_along_axis(cand, part, axis=1)
    tracks = [picked[j, :t[j]] for j in range(m)]
    return _finish(rng, cams, pts, tracks, f"spiral_slab_n{n}", seed, with_info)


def _zipf_lengths(rng, m, s=1.5, lo=2, hi=30):
    k = np.arange(lo, hi + 1)
    p = k ** (-s)
    p /= p.sum()
    return rng.choice(k, size=m, p=p)


def clustered(seed: int = 0, n_clusters: int = 10, per_cluster: int = 300,
              m: int = 500_000, ring: float = 40.0, frac_cross: float = 0.02,
              frac_far: float = 0.05, with_info: bool = False, max_track: int = 30) -> Scene:
    """Clustered sites: n_clusters groups of per_cluster cameras, each group
    on a ring of radius 12 (heights 1-5) around its own object (points in a
    cylinder of radius 4, height [-2, 2]) at a site on a circle of radius
    ``ring``.  Track lengths Zipf(1.5) on [2, max_track], capped by the
    cameras that see the point inside the 640 x 480 frame; a track is the arc
    of cameras nearest a random seeing camera among those that see it.
    ``frac_cross`` of the points lie between neighbouring sites and are seen
    from both (half the track each), which links the sites; ``frac_far`` lie
    about 1000 units away along a camera's viewing ray and are seen by its
    neighbours, a near-zero baseline that makes their 3 x 3 point blocks
    ill-conditioned.  Every observed point is in front of its cameras."""
    rng = np.random.default_rng(seed)
    n = n_clusters * per_cluster
    ang = 2 * np.pi * np.arange(n_clusters) / n_clusters
    site = ring * np.column_stack([np.cos(ang), np.sin(ang), np.zeros(n_clusters)])
    cl = np.repeat(np.arange(n_clusters), per_cluster)
    phi = (2 * np.pi * np.tile(np.arange(per_cluster), n_clusters) / per_cluster
           + rng.normal(0.0, 0.3 * np.pi / per_cluster, n))
    centres = site[cl] + np.column_stack([12.0 * np.cos(phi), 12.0 * np.sin(phi),
                                          rng.uniform(1.0, 5.0, n)])
    target = site[cl] + rng.normal(0.0, 0.5, (n, 3))
    axes = _look_at_axes(target - centres, np.tile([0.0, 0.0, 1.0], (n, 1)))
    cams = np.column_stack([Rotation.from_matrix(axes).as_rotvec(), centres, _intrinsics(rng, n)])
    members = [np.flatnonzero(cl == c) for c in range(n_clusters)]
    kind = rng.uniform(0, 1, m)
    n_cross = int((kind < frac_cross).sum())
    n_far = int(((kind >= frac_cross) & (kind < frac_cross + frac_far)).sum())
    n_local = m - n_cross - n_far

    def draw_tracks(P, cand, want, chunk=4096):
        # per point: the candidates that see it, then the arc of the t nearest
        # to a random one of them (None when fewer than two see it)
        out = []
        for j0 in range(0, P.shape[0], chunk):
            Pc, cc = P[j0:j0 + chunk], cand[j0:j0 + chunk]
            vis = _in_view(axes, centres, Pc, cc)
            nvis = vis.sum(axis=1)
            keys = rng.random(vis.shape)
            keys[~vis] = np.inf
            anchor = centres[cc[np.arange(cc.shape[0]), np.argmin(keys, axis=1)]]
            dist = np.linalg.norm(centres[cc] - anchor[:, None, :], axis=2)
            dist[~vis] = np.inf
            order = np.argsort(dist, axis=1, kind="stable")
            t = np.minimum(want[j0:j0 + chunk], nvis)
            for q in range(cc.shape[0]):
                out.append(cc[q, order[q, :t[q]]] if nvis[q] >= 2 else None)
        return out

    pts_l, tracks = [], []
    # local points of every site
    per_site = np.bincount(rng.integers(0, n_clusters, n_local), minlength=n_clusters)
    for c in range(n_clusters):
        need = int(per_site[c])
        while need > 0:
            b = int(1.2 * need) + 16
            r = 4.0 * np.sqrt(rng.uniform(0, 1, b))
            th = rng.uniform(0, 2 * np.pi, b)
            P = site[c] + np.column_stack([r * np.cos(th), r * np.sin(th), rng.uniform(-2, 2, b)])
            cand = np.tile(members[c], (b, 1))
            tr = draw_tracks(P, cand, _zipf_lengths(rng, b, hi=max_track))
            for j in range(b):
                if tr[j] is not None and need > 0:
                    pts_l.append(P[j])
                    tracks.append(tr[j])
                    need -= 1
    # points between neighbouring sites, seen from both
    need = n_cross
    while need > 0:
        b = int(2 * need) + 16
        c = rng.integers(0, n_clusters, b)
        d = (c + 1) % n_clusters
        P = 0.5 * (site[c] + site[d]) + np.column_stack([rng.normal(0, 3.0, (b, 2)),
                                                         rng.uniform(0.0, 4.0, b)])
        want = _zipf_lengths(rng, b, hi=max_track)
        ta = np.maximum(1, want // 2)
        tb = np.maximum(1, want - ta)
        tr_a = draw_tracks(P, np.stack([members[x] for x in c]), 2 * ta)
        tr_b = draw_tracks(P, np.stack([members[x] for x in d]), 2 * tb)
        for j in range(b):
            if tr_a[j] is None or tr_b[j] is None or need == 0:
                continue
            pts_l.append(P[j])
            tracks.append(np.concatenate([tr_a[j][:ta[j]], tr_b[j][:tb[j]]]))
            need -= 1
    # far points: near-zero baseline
    need = n_far
    while need > 0:
        b = int(1.2 * need) + 16
        a = rng.integers(0, n, b)
        ray = np.column_stack([rng.uniform(-0.25, 0.25, b), rng.uniform(-0.18, 0.18, b), np.ones(b)])
        ray = (axes[a] * ray[:, :, None]).sum(axis=1)
        ray /= np.linalg.norm(ray, axis=1, keepdims=True)
        P = centres[a] + ray * rng.uniform(800.0, 1200.0, b)[:, None]
        cand = np.stack([members[x] for x in cl[a]])
        tr = draw_tracks(P, cand, _zipf_lengths(rng, b, hi=max_track))
        for j in range(b):
            if tr[j] is not None and need > 0:
                pts_l.append(P[j])
                tracks.append(tr[j])
                need -= 1
    pts = np.asarray(pts_l)
    order = rng.permutation(len(tracks))
    return _finish(rng, cams, pts[order], [tracks[i] for i in order], "clustered", seed, with_info)


def batch_scenes(seed: int = 1000, count: int = 256, lo: int = 20, hi: int = 400,
                 pts_per_cam: int = 100, p_geom: float = 0.25) -> list[Scene]:
    """Independent sub-reconstructions with log-uniform camera counts."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(int)
    out = []
    for s, n in enumerate(sizes):
        # a stretch of the 500-camera spiral: the same camera spacing and
        # height, so neighbouring views overlap as much as there
        out.append(spiral_slab(seed + 1 + s, n=int(n), m=int(pts_per_cam * n),
                               p_geom=p_geom, turns=3.0 * n / 500.0))
    return out


def by_name(name: str, seed: int = 0) -> Scene:
    if name == "tiny_circle":
        return tiny_circle(seed)
    if name == "spiral_slab":
        return spiral_slab(seed)
    if name == "clustered":
        return clustered(seed)
    raise KeyError(name)


def mlp_init(seed: int, layers=(55, 256, 256, 256, 45)) -> np.ndarray:
    """Initial parameters of a ReLU MLP as one flat float64 vector: for each
    layer W (out x in, row-major, N(0, 2/in)) followed by b (zeros)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in zip(layers[:-1], layers[1:]):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / i), o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def additions(scene: Scene, seed: int, k: int, new_camera: bool = False):
    """Seeded new observations for incremental updates.  Without new_camera:
    k pairs (camera, point) not yet observed, the camera a spiral/ring
    neighbour (index within 3) of one of the point's cameras with the point in
    front of it.  With new_camera: a new camera, a perturbed copy of a random
    camera, observing up to k of the points its source sees that lie in front
    of it.  Returns (new_cam, new_pt, new_info or None, cam_new or None); the
    new camera has index n_cams."""
    rng = np.random.default_rng(seed)
    n, m = scene.n_cams, scene.n_pts

    def in_front(cam, X):
        R = Rotation.from_rotvec(cam[0:3]).as_matrix()
        return float((R @ (X - cam[3:6]))[2]) > 0.0

    if new_camera:
        src = int(rng.integers(n))
        cam_new = scene.cams[src].copy()
        spread = float(np.linalg.norm(scene.cams[:, 3:6].std(axis=0)))
        cam_new[3:6] += rng.normal(0.0, 0.02 * spread, 3)
        cam_new[0:3] += rng.normal(0.0, 0.01, 3)
        pts = [int(j) for j in scene.obs_pt[scene.obs_cam == src] if in_front(cam_new, scene.pts[j])]
        sel = rng.choice(len(pts), size=min(k, len(pts)), replace=False)
        pt = np.sort(np.asarray([pts[q] for q in sel], np.int32))
        info = None if scene.obs_info is None else random_information(rng, pt.size)
        return np.full(pt.size, n, np.int32), pt, info, cam_new
    seen = set(zip(scene.obs_cam.tolist(), scene.obs_pt.tolist()))
    cams_of = {}
    for c, j in zip(scene.obs_cam.tolist(), scene.obs_pt.tolist()):
        cams_of.setdefault(j, []).append(c)
    cam, pt = [], []
    tries = 0
    while len(cam) < k and tries < 100 * k:
        tries += 1
        j = int(rng.integers(m))
        c0 = cams_of[j][int(rng.integers(len(cams_of[j])))]
        c = (c0 + int(rng.integers(-3, 4))) % n
        if (c, j) in seen or not in_front(scene.cams[c], scene.pts[j]):
            continue
        seen.add((c, j))
        cam.append(c)
        pt.append(j)
    info = None if scene.obs_info is None else random_information(rng, len(cam))
    return np.asarray(cam, np.int32), np.asarray(pt, np.int32), info, None


def view_graph_partition(scene: Scene, k: int, seed: int, min_shared: int = 8,
                         min_support: int = 10) -> np.ndarray:
    """Group ids (n_cams,) of a decomposition into groups of about k cameras
    whose sub-reconstructions are well posed.

    Two cameras are strongly linked when they share at least ``min_shared``
    points.  round(n / k) seeds are spread over the view graph (a seeded
    random camera, then each time a camera farthest in strong-link hops from
    all seeds so far); the groups then grow together, in turn, each adding
    the unassigned camera with the most points shared with it along strong
    links.  A group left smaller than k / 2 joins the strongly linked
    neighbour it shares most points with.  Then, until nothing changes, every
    group registers its cameras as incremental reconstruction would (the
    pair sharing most points first, then any camera that sees at least
    ``min_support`` points already seen by two registered cameras), and a
    camera left unregistered moves to the neighbouring group whose
    registered cameras fix more of its points.  A camera attached to its
    group only through points it shares with a single other camera, or a
    chain of cameras hanging from one camera, would leave the length of a
    baseline free: the sub-reconstruction would have a null space larger
    than the similarity gauge.  Used as the decomposition input of
    sub-reconstruction runs."""
    n = scene.n_cams
    oc, op = scene.obs_cam.astype(np.int64), scene.obs_pt.astype(np.int64)
    by_pt = {}
    for c, j in zip(oc.tolist(), op.tolist()):
        by_pt.setdefault(j, []).append(c)
    adj = [dict() for _ in range(n)]
    for cams in by_pt.values():
        for a in cams:
            for b in cams:
                if a != b:
                    adj[a][b] = adj[a].get(b, 0) + 1
    strong = [{b: w for b, w in adj[a].items() if w >= min_shared} for a in range(n)]
    cam_pts = [[] for _ in range(n)]
    for c, j in zip(oc.tolist(), op.tolist()):
        cam_pts[c].append(j)
    rng = np.random.default_rng(seed)
    group = np.full(n, -1, dtype=np.int64)
    # seeds: a random camera, then repeatedly the camera farthest (in hops
    # along strong links) from every seed so far
    n_groups = max(1, int(round(n / k)))
    hops = np.full(n, np.iinfo(np.int64).max, dtype=np.int64)
    seeds = []
    nxt_seed = int(rng.integers(n))
    for _ in range(n_groups):
        seeds.append(nxt_seed)
        hops[nxt_seed] = 0
        frontier = [nxt_seed]
        d = 0
        while frontier:
            d += 1
            new = []
            for a in frontier:
                for b in strong[a]:
                    if hops[b] > d:
                        hops[b] = d
                        new.append(b)
            frontier = new
        far = np.flatnonzero(hops == hops.max())
        nxt_seed = int(far[rng.integers(far.size)])
    # all groups grow together, one camera per group in turn, each taking the
    # unassigned camera that shares the most points with it along strong links
    scores = [{} for _ in seeds]
    sizes = [0] * len(seeds)

    def take(gid, c):
        group[c] = gid
        sizes[gid] += 1
        for b, w in strong[c].items():
            if group[b] < 0:
                scores[gid][b] = scores[gid].get(b, 0) + w

    for gid, c in enumerate(seeds):
        take(gid, c)
    active = True
    while active:
        active = False
        for gid in range(len(seeds)):
            sc = scores[gid]
            while sc:
                c, _ = max(sc.items(), key=lambda kv: (kv[1], -kv[0]))
                del sc[c]
                if group[c] < 0:
                    take(gid, c)
                    active = True
                    break
    # cameras no strong link reaches start groups of their own
    for c in np.flatnonzero(group < 0).tolist():
        if group[c] < 0:
            sizes.append(0)
            scores.append({})
            gid = len(sizes) - 1
            take(gid, c)
            while scores[gid] and sizes[gid] < k:
                b, _ = max(scores[gid].items(), key=lambda kv: (kv[1], -kv[0]))
                del scores[gid][b]
                if group[b] < 0:
                    take(gid, b)

    def links_of(cams, own):
        links = {}
        for a in cams:
            for b, w in adj[a].items():
                if group[b] != own:
                    links[group[b]] = links.get(group[b], 0) + w
        return links

    for gid, size in enumerate(sizes):
        if size >= max(2, k // 2):
            continue
        mine = np.flatnonzero(group == gid).tolist()
        links = links_of(mine, gid)
        if links:
            group[mine] = max(links.items(), key=lambda kv: (kv[1], -kv[0]))[0]

    def rigid_core(members):
        # cameras registered as in incremental reconstruction: the pair that
        # shares most points, then repeatedly the camera that sees the most
        # points already seen by two registered cameras, while it sees at
        # least min_support of them
        mem = set(members)
        pair = max(((w, a, b) for a in members for b, w in adj[a].items() if b in mem and a < b),
                   default=None)
        if pair is None:
            return set(), set()
        core = set()
        seen, fixed, cnt = {}, set(), {c: 0 for c in members}

        def register(c):
            core.add(c)
            for j in cam_pts[c]:
                seen[j] = seen.get(j, 0) + 1
                if seen[j] == 2:
                    fixed.add(j)
                    for b in by_pt[j]:
                        if b in mem and b not in core:
                            cnt[b] += 1

        register(pair[1])
        register(pair[2])
        while True:
            rest = [c for c in members if c not in core]
            if not rest:
                break
            c = max(rest, key=lambda c: (cnt[c], -c))
            if cnt[c] < min_support:
                break
            register(c)
        return core, fixed

    for _ in range(20):
        changed = False
        gids = np.unique(group).tolist()
        cores = {g: rigid_core(np.flatnonzero(group == g).tolist()) for g in gids}
        for g in gids:
            core, _ = cores[g]
            for c in np.flatnonzero(group == g).tolist():
                if c in core:
                    continue
                own = sum(1 for j in cam_pts[c] if j in cores[g][1])
                cand = {group[b] for b in adj[c]} - {g}
                best = max(cand, key=lambda h: (sum(1 for j in cam_pts[c] if j in cores[h][1]), -h),
                           default=None)
                if best is not None and sum(1 for j in cam_pts[c] if j in cores[best][1]) > own:
                    group[c] = best
                    changed = True
        if not changed:
            break
    _, dense = np.unique(group, return_inverse=True)
    return dense.astype(np.int32)

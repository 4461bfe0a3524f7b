"""Seeded synthetic inputs for cone-beam backprojection.

This module only *makes inputs*: C-arm projection matrices, an ellipsoid phantom,
its exact line integrals, and the host-side FDK preprocessing (cosine weight,
Parker short-scan weight, ramp filter) that turns line integrals into the
filtered projections the backprojector consumes.  It contains no
backprojection arithmetic; the FP64 oracle and the GPU library both receive
the arrays produced here and nothing else is shared between them.

Stand-in for the paper's workload: the paper backprojects a proprietary C-arm
rabbit scan (496 filtered FP32 projections of 1248x960, one 3x4 matrix each,
Sec. "RabbitCT Benchmarking Framework").  That dataset is not available, so the
same shapes are produced from a seeded analytic phantom.

Conventions (shared by every consumer of these arrays):
  * matrices are FP64, shape (N, 3, 4), row-major P[r][c]; a world point X (mm)
    maps to homogeneous detector coordinates (u, v, w) = P @ (X, 1) and to the
    pixel (u / w, v / w); pixel (i, j) is centred on integer coordinates;
  * projections are (N, H, W) with the column index i (u) fastest;
  * the scan is a circular short scan over ``arc_deg`` degrees about the z axis
    with equal steps, theta_k = k * arc / (N - 1), source at
    SID * (cos theta, sin theta, 0); w is the depth along the central ray in mm.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

__all__ = [
    "CArm", "carm_matrices", "Phantom", "ellipsoid_phantom", "project_phantom",
    "fdk_filter", "voxelize_phantom", "filtered_projections", "random_projections",
    "tiny_cone_matrices", "default_origin", "ScanSpec", "batched_scan_specs",
]


@dataclass(frozen=True)
class CArm:
    """Circular short-scan C-arm: all lengths in mm, angles in degrees."""
    n_proj: int
    width: int = 1248
    height: int = 960
    sid: float = 750.0      # source to isocentre
    sdd: float = 1200.0     # source to detector
    pixel: float = 0.308    # detector pixel pitch
    arc_deg: float = 200.0  # short-scan arc
    tilt_deg: float = 0.0   # camera frame tilted about its u axis (0: the orbit plane is the mid-plane)

    @property
    def focal_px(self) -> float:
        return self.sdd / self.pixel

    @property
    def principal_point(self) -> tuple[float, float]:
        return ((self.width - 1) / 2.0, (self.height - 1) / 2.0)

    def angles_rad(self) -> np.ndarray:
        if self.n_proj == 1:
            return np.zeros(1)
        k = np.arange(self.n_proj, dtype=np.float64)
        return np.deg2rad(k * self.arc_deg / (self.n_proj - 1))


def carm_matrices(carm: CArm) -> np.ndarray:
    """Projection matrices P_k = K [R_k | t_k] in FP64, shape (N, 3, 4).

    Camera frame: x_cam = e_u (tangential, the direction the source moves),
    y_cam = (0, 0, -1) (detector rows run along -z), z_cam = e_d (from the
    source towards the isocentre); with tilt_deg the camera frame is turned
    about x_cam, so the depth axis leaves the orbit plane (as in calibrated
    real C-arms) and w depends on z.  The third row of [R|t] has unit norm, so
    w is the source-to-voxel depth along the central ray in mm.
    """
    f = carm.focal_px
    cu, cv = carm.principal_point
    K = np.array([[f, 0.0, cu], [0.0, f, cv], [0.0, 0.0, 1.0]])
    mats = np.empty((carm.n_proj, 3, 4))
    for k, th in enumerate(carm.angles_rad()):
        c, s = math.cos(th), math.sin(th)
        src = carm.sid * np.array([c, s, 0.0])
        R = np.array([[-s, c, 0.0], [0.0, 0.0, -1.0], [-c, -s, 0.0]])
        if carm.tilt_deg != 0.0:
            ct, st = math.cos(math.radians(carm.tilt_deg)), math.sin(math.radians(carm.tilt_deg))
            R = np.array([[1.0, 0.0, 0.0], [0.0, ct, -st], [0.0, st, ct]]) @ R
        t = -R @ src
        mats[k] = K @ np.concatenate([R, t[:, None]], axis=1)
    return mats


def default_origin(L: int, voxel_mm: float) -> tuple[float, float, float]:
    """Centre of voxel 0 when the volume is centred on the isocentre."""
    o = -(L - 1) * voxel_mm / 2.0
    return (o, o, o)


@dataclass
class Phantom:
    centres: np.ndarray   # (n, 3) mm
    axes: np.ndarray      # (n, 3) semi-axes, mm
    rot: np.ndarray       # (n, 3, 3), columns are the ellipsoid's axes in world frame
    rho: np.ndarray       # (n,) density (1/mm: line integrals are in units of rho*mm)
    seed: int = 0


def ellipsoid_phantom(seed: int, n: int = 10, semi_axes=(5.0, 60.0),
                      centre_box=(40.0, 40.0, 30.0)) -> Phantom:
    """Seeded random ellipsoids: semi-axes U[5, 60] mm, densities U[0, 1],
    centres uniform in [-40, 40]^2 x [-30, 30] mm, orientation from a seeded
    unit quaternion.  Overlapping ellipsoids add."""
    rng = np.random.default_rng(seed)
    box = np.asarray(centre_box)
    centres = rng.uniform(-box, box, size=(n, 3))
    axes = rng.uniform(semi_axes[0], semi_axes[1], size=(n, 3))
    rho = rng.uniform(0.0, 1.0, size=n)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    a, b, c, d = q.T
    rot = np.stack([
        np.stack([a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)], -1),
        np.stack([2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)], -1),
        np.stack([2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d], -1),
    ], axis=1)
    return Phantom(centres, axes, rot, rho, seed)


def project_phantom(mats: np.ndarray, width: int, height: int, ph: Phantom,
                    device="cpu") -> torch.Tensor:
    """Exact line integrals of the phantom through every pixel centre, FP64.

    For P = [M | p4] the source is C = -M^-1 p4 and the ray through pixel
    (i, j) has direction M^-1 (i, j, 1).  In an ellipsoid's unit-sphere frame
    (o', d') the chord length of the unit-speed line is 2 sqrt(B^2 - A C) / A
    with A = d'.d', B = o'.d', C = o'.o' - 1.
    """
    dev = torch.device(device)
    N = mats.shape[0]
    out = torch.zeros((N, height, width), dtype=torch.float64, device=dev)
    jj, ii = torch.meshgrid(torch.arange(height, dtype=torch.float64, device=dev),
                            torch.arange(width, dtype=torch.float64, device=dev), indexing="ij")
    pix = torch.stack([ii, jj, torch.ones_like(ii)], dim=-1).reshape(-1, 3)  # (HW, 3)
    cen = torch.as_tensor(ph.centres, device=dev)
    inv_a = torch.as_tensor(1.0 / ph.axes, device=dev)
    rotT = torch.as_tensor(ph.rot, device=dev).transpose(1, 2)  # world -> ellipsoid frame
    rho = torch.as_tensor(ph.rho, device=dev)
    # a batch of projections at a time (about 2^24 rays)
    nb = max(1, (1 << 24) // (height * width))
    for k0 in range(0, N, nb):
        ks = range(k0, min(N, k0 + nb))
        Minv = np.stack([np.linalg.inv(mats[k, :, :3]) for k in ks])                       # (b, 3, 3)
        C = torch.as_tensor(np.stack([-Minv[i] @ mats[k, :, 3] for i, k in enumerate(ks)]), device=dev)  # (b, 3)
        d = torch.einsum("pc,brc->bpr", pix, torch.as_tensor(Minv, device=dev))          # (b, HW, 3)
        d = d / torch.linalg.norm(d, dim=2, keepdim=True)
        acc = torch.zeros(d.shape[:2], dtype=torch.float64, device=dev)
        for e in range(len(ph.rho)):
            o = ((C - cen[e]) @ rotT[e].T) * inv_a[e]                                       # (b, 3)
            de = (d @ rotT[e].T) * inv_a[e]                                                 # (b, HW, 3)
            A = (de * de).sum(2)
            B = (de * o[:, None, :]).sum(2)
            Cc = (o * o).sum(1, keepdim=True) - 1.0
            disc = B * B - A * Cc
            acc += torch.where(disc > 0, 2.0 * torch.sqrt(disc.clamp_min(0)) / A, 0.0) * rho[e]
        out[k0:k0 + len(ks)] = acc.reshape(len(ks), height, width)
    return out


def _ramp_kernel(n: int, tau: float, dev) -> torch.Tensor:
    """Band-limited ramp filter sampled at spacing tau (Kak & Slaney):
    h(0) = 1/(4 tau^2), h(even) = 0, h(odd n) = -1/(n pi tau)^2; length 2n-1
    laid out circularly for an FFT of size >= 2n."""
    size = 1 << int(math.ceil(math.log2(2 * n)))
    idx = torch.arange(size, device=dev)
    nn = torch.where(idx < size // 2, idx, idx - size).to(torch.float64)
    h = torch.zeros(size, dtype=torch.float64, device=dev)
    odd = (nn.abs() % 2) == 1
    h[odd] = -1.0 / (nn[odd] * math.pi * tau) ** 2
    h[0] = 1.0 / (4.0 * tau * tau)
    return h


def fdk_filter(lineint: torch.Tensor, carm: CArm) -> torch.Tensor:
    """FDK preprocessing of line integrals (N, H, W) -> filtered projections.

    Cosine weight SDD / sqrt(SDD^2 + u^2 + v^2); Parker short-scan weight
    (Parker 1982, with overscan delta = (arc - pi) / 2 >= fan half-angle);
    ramp filter along detector rows at the isocentre pitch tau = pixel*SID/SDD;
    the constants (d_beta, SID^2) are folded in so that the backprojection
    sum_k p_k(u/w, v/w) / w^2 estimates the density.
    """
    dev = lineint.device
    N, H, W = lineint.shape
    cu, cv = carm.principal_point
    u = (torch.arange(W, dtype=torch.float64, device=dev) - cu) * carm.pixel
    v = (torch.arange(H, dtype=torch.float64, device=dev) - cv) * carm.pixel
    cosw = carm.sdd / torch.sqrt(carm.sdd ** 2 + u[None, :] ** 2 + v[:, None] ** 2)
    arc = math.radians(carm.arc_deg)
    delta = (arc - math.pi) / 2.0
    gam = -torch.atan(u / carm.sdd)   # fan angle in the sense of increasing theta
    gmax = math.atan((W / 2.0) * carm.pixel / carm.sdd)
    if delta < gmax:
        raise ValueError("arc too short for a Parker short scan")
    beta = torch.as_tensor(carm.angles_rad(), device=dev)[:, None]
    g = gam[None, :]
    w1 = torch.sin(math.pi / 4 * beta / (delta - g)) ** 2
    w3 = torch.sin(math.pi / 4 * (math.pi + 2 * delta - beta) / (delta + g)) ** 2
    parker = torch.where(beta < 2 * delta - 2 * g, w1,
                         torch.where(beta <= math.pi - 2 * g, torch.ones_like(w1), w3))
    parker = torch.where((beta < 0) | (beta > math.pi + 2 * delta), 0.0, parker)
    x = lineint * cosw[None] * parker[:, None, :]
    tau = carm.pixel * carm.sid / carm.sdd
    h = _ramp_kernel(W, tau, dev)
    size = h.numel()
    Hf = torch.fft.rfft(h)
    X = torch.fft.rfft(x, n=size, dim=-1)
    q = torch.fft.irfft(X * Hf, n=size, dim=-1)[..., :W] * tau
    dbeta = arc / (N - 1) if N > 1 else arc
    return q * (dbeta * carm.sid ** 2)


def filtered_projections(carm: CArm, seed: int, device="cpu") -> tuple[np.ndarray, torch.Tensor]:
    """Matrices and FP32 filtered projections of the seeded phantom."""
    mats = carm_matrices(carm)
    ph = ellipsoid_phantom(seed)
    li = project_phantom(mats, carm.width, carm.height, ph, device)
    q = fdk_filter(li, carm).to(torch.float32)
    del li
    return mats, q


def voxelize_phantom(ph: Phantom, L: int, voxel_mm: float, origin=None,
                     device="cpu") -> torch.Tensor:
    """Centre-sampled density of the phantom on the L^3 grid, index (z, y, x)."""
    dev = torch.device(device)
    o = default_origin(L, voxel_mm) if origin is None else origin
    ax = [o[a] + voxel_mm * torch.arange(L, dtype=torch.float64, device=dev) for a in range(3)]
    Z, Y, X = torch.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    P = torch.stack([X, Y, Z], -1)
    out = torch.zeros((L, L, L), dtype=torch.float64, device=dev)
    for e in range(len(ph.rho)):
        q = ((P - torch.as_tensor(ph.centres[e], device=dev)) @ torch.as_tensor(ph.rot[e], device=dev))
        q = q / torch.as_tensor(ph.axes[e], device=dev)
        out += torch.where((q * q).sum(-1) <= 1.0, float(ph.rho[e]), 0.0)
    return out


def random_projections(n: int, h: int, w: int, seed: int, dist="normal") -> np.ndarray:
    """Seeded FP32 projection stack (N, H, W)."""
    rng = np.random.default_rng(seed)
    if dist == "normal":
        return rng.standard_normal((n, h, w), dtype=np.float32)
    return rng.uniform(-1.0, 1.0, size=(n, h, w)).astype(np.float32)


def tiny_cone_matrices(n: int, width: int, height: int, L: int, voxel_mm: float,
                       seed: int, jitter: float = 0.02) -> np.ndarray:
    """Perspective matrices for tiny brute-force cases: a C-arm whose detector
    pitch is chosen so that an L^3 volume of the given voxel size overfills the
    small detector (some voxels project off it, some onto its edges), with a
    seeded relative jitter of every entry so no symmetry hides an index error."""
    rng = np.random.default_rng(seed)
    half = (L - 1) * voxel_mm / 2.0
    sid = 20.0 * max(half, voxel_mm)
    sdd = 1.6 * sid
    # detector spans roughly 80% of the magnified volume
    pixel = 0.8 * (2 * half * sdd / sid) / max(width, 2)
    carm = CArm(n, width, height, sid=sid, sdd=sdd, pixel=pixel, arc_deg=200.0)
    mats = carm_matrices(carm)
    mats = mats * (1.0 + jitter * rng.uniform(-1, 1, size=mats.shape))
    return mats


@dataclass
class ScanSpec:
    """One scan of the batched workload."""
    L: int
    voxel_mm: float
    n_proj: int
    width: int
    height: int
    pixel: float
    sid: float
    seed: int

    def carm(self) -> CArm:
        return CArm(self.n_proj, self.width, self.height, sid=self.sid, sdd=1200.0,
                    pixel=self.pixel, arc_deg=200.0)


def batched_scan_specs(n_scans: int = 16, seed: int = 100) -> list[ScanSpec]:
    """Uneven scans: L in {64, 96, 128, 192, 256}, N in {124, 248, 496},
    detector 1248x960 @ 0.308 mm or 620x480 @ 0.616 mm, SID U[600, 800] mm,
    SDD 1200 mm, 0.5 mm voxels, phantom seeds seed, seed+1, ..."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_scans):
        L = int(rng.choice([64, 96, 128, 192, 256]))
        N = int(rng.choice([124, 248, 496]))
        big = bool(rng.integers(0, 2))
        W, H, pix = (1248, 960, 0.308) if big else (620, 480, 0.616)
        sid = float(rng.uniform(600.0, 800.0))
        out.append(ScanSpec(L, 0.5, N, W, H, pix, sid, seed + i))
    return out


def batched_phantom_scans(specs: list[ScanSpec], device="cpu") -> list[tuple[np.ndarray, torch.Tensor]]:
    """Matrices and FP32 filtered projections of every scan's own seeded
    phantom (seed = spec.seed), on that scan's C-arm."""
    return [filtered_projections(sp.carm(), sp.seed, device=device) for sp in specs]


def xxl_carm(n_proj: int) -> CArm:
    """A large industrial cone-beam scanner with a 10000 x 10000 detector
    (381 MiB per FP32 projection): SID 2000 mm, SDD 3000 mm, 0.15 mm pixels
    (1.5 m detector, 1 m field at the isocentre), short scan of 210 degrees
    (fan half-angle 14.0 degrees).  A 0.25 mm voxel then spans 2.5 pixels at
    the isocentre, as a 0.5 mm voxel does on the 1248 x 960 C-arm."""
    return CArm(n_proj, 10000, 10000, sid=2000.0, sdd=3000.0, pixel=0.15, arc_deg=210.0)

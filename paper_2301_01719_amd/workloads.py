"""Seeded synthetic inputs for the radiance-bucket lookup.

This module generates inputs only: textures, G-buffers (UV, tangent frame,
view vector) and upstream gradients.  It holds none of the lookup's own
arithmetic, so both the GPU path and the CPU oracle can consume what it
produces.  Random numbers come from one counter-based generator (the
SplitMix64 finaliser of Steele, Lea and Flood, 2014, applied to
index * golden-gamma + key(seed, stream)), so the same (seed, stream, index)
gives the same number on any device and for any thread count.

Workloads (bucket matrix W x H of n x n samples with C channels):
  C1  64x64 buckets, n=8, RGBA f32, texels i.i.d. U[0,1); 256x256 fragments,
      UV i.i.d. U[0,1)^2, identity frame, views uniform on the cap of the
      upper hemisphere with elevation >= 5 degrees.
  C2  1024x1024 buckets, n=16, RGBA, smooth radiance; one 1920x1080 view of
      a perspective camera over a UV-tiled plane, normals perturbed by
      N(0, 10 deg).
  C3  512x512 buckets, n=16, RGBA, smooth radiance; 64 views of 1024x1024.
  C4  256x256 buckets, n=8, RGB, smooth radiance; 16 views of 512x512.
  C5  2048x2048 buckets, n=16, RGBA, smooth radiance; 8 views of 3840x2160
      over a bumpy height field (gradient noise, amplitude 0.1).

Shadow scenes (Sec. 5, Shadowing): balls hovering over the UV-tiled plane
z = 0 stand in for static occluders; lights are sets of directions (a sun
disc) or points (a spherical lamp), sampled on golden-angle spirals.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Tuple

import torch

_M64 = (1 << 64) - 1


def _s64(c: int) -> int:
    c &= _M64
    return c - (1 << 64) if c >= (1 << 63) else c


_GOLDEN = _s64(0x9E3779B97F4A7C15)
_K1 = _s64(0xBF58476D1CE4E5B9)
_K2 = _s64(0x94D049BB133111EB)

# stream ids
S_TEXTURE, S_CAMERA, S_UV, S_VIEW, S_NORMAL, S_GRAD, S_NOISE, S_BALLS = 0, 1, 2, 3, 4, 5, 6, 7


def _mix_py(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    return (x >> k) & ((1 << (64 - k)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _K1
    z = (z ^ _srl(z, 27)) * _K2
    return z ^ _srl(z, 31)


def _bits(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    key = _s64(_mix_py((seed << 24) ^ (stream << 8) ^ 0x5A5A))
    return _mix(idx.to(torch.int64) * _GOLDEN + key)


def uniform(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """float32 uniforms k / 2^24 in [0, 1) for an int64 index tensor."""
    z = _bits(seed, stream, idx)
    return _srl(z, 40).to(torch.float32) * (1.0 / 16777216.0)


def uniform64(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """float64 uniforms k / 2^53 in [0, 1)."""
    z = _bits(seed, stream, idx)
    return _srl(z, 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def _arange(n: int, device) -> torch.Tensor:
    return torch.arange(n, dtype=torch.int64, device=device)


def normal_pair(seed: int, stream: int, n: int, device, offset: int = 0):
    """Two independent N(0,1) float64 tensors of length n (Box-Muller)."""
    i = _arange(n, device) + offset
    u1 = uniform64(seed, stream, 2 * i)
    u2 = uniform64(seed, stream, 2 * i + 1)
    r = torch.sqrt(-2.0 * torch.log1p(-u1))
    t = 2.0 * math.pi * u2
    return r * torch.cos(t), r * torch.sin(t)


# ---------------------------------------------------------------------------
# textures (bucket-major [H][W][n][n][C] float32)
# ---------------------------------------------------------------------------

def iid_texture(W: int, H: int, n: int, C: int, seed: int, device="cpu") -> torch.Tensor:
    total = W * H * n * n * C
    return uniform(seed, S_TEXTURE, _arange(total, device)).reshape(H, W, n, n, C)


def smooth_texture(W: int, H: int, n: int, C: int, seed: int, device="cpu",
                   terms: int = 8) -> torch.Tensor:
    """Smooth radiance: per channel clamp(0.5 + sum_k a_k sin(2 pi (p_k U + q_k V)
    + alpha_k b_x + beta_k b_y + phi_k), 0, 1), with (U, V) the bucket centre in
    UV and (b_x, b_y) the sample centre in [-1, 1]^2.  p_k, q_k are integers in
    [-8, 8] so the texture repeats seamlessly under UV wrap.  Evaluated with the
    separable identity sin(P + Q) = sin P cos Q + cos P sin Q as one small
    matrix product per channel."""
    K = terms
    prm = uniform64(seed, S_TEXTURE, _arange(C * K * 6, "cpu")).reshape(C, K, 6)
    U = (torch.arange(W, dtype=torch.float64, device=device) + 0.5) / W
    V = (torch.arange(H, dtype=torch.float64, device=device) + 0.5) / H
    bx = (2.0 * torch.arange(n, dtype=torch.float64, device=device) + 1.0) / n - 1.0
    out = torch.empty((H * W, n * n, C), dtype=torch.float32, device=device)
    for c in range(C):
        p = torch.floor(prm[c, :, 0] * 17.0) - 8.0
        q = torch.floor(prm[c, :, 1] * 17.0) - 8.0
        al = (prm[c, :, 2] * 2.0 - 1.0) * math.pi
        be = (prm[c, :, 3] * 2.0 - 1.0) * math.pi
        ph = prm[c, :, 4] * 2.0 * math.pi
        amp = prm[c, :, 5] * 0.25
        p, q, al, be, ph, amp = (t.to(device) for t in (p, q, al, be, ph, amp))
        # bucket table P[j, i, k]
        P = (2.0 * math.pi * (p[None, None, :] * U[None, :, None]
                              + q[None, None, :] * V[:, None, None]) + ph)
        P = P.reshape(H * W, K)
        left = torch.cat([torch.sin(P) * amp, torch.cos(P) * amp], dim=1).to(torch.float32)
        del P
        # sample table Q[y, x, k]
        Q = al[None, None, :] * bx[None, :, None] + be[None, None, :] * bx[:, None, None]
        Q = Q.reshape(n * n, K)
        right = torch.cat([torch.cos(Q), torch.sin(Q)], dim=1).to(torch.float32)
        val = torch.matmul(left, right.t().contiguous())
        val.add_(0.5).clamp_(0.0, 1.0)
        out[:, :, c] = val
        del val, left
    return out.reshape(H, W, n, n, C)


# ---------------------------------------------------------------------------
# G-buffers
# ---------------------------------------------------------------------------

def _frame_from_normal(Nv: torch.Tensor) -> torch.Tensor:
    """Rows (T, B, N) with T = normalize(e_x - (e_x . N) N), B = N x T."""
    ex = torch.zeros_like(Nv)
    ex[..., 0] = 1.0
    T = ex - (Nv[..., 0:1]) * Nv
    T = T / torch.linalg.vector_norm(T, dim=-1, keepdim=True)
    B = torch.linalg.cross(Nv, T, dim=-1)
    return torch.stack([T, B, Nv], dim=-2)


@dataclass
class GBuffer:
    uv: torch.Tensor    # [N, 2] float32
    tbn: torch.Tensor   # [N, 3, 3] float32, rows T, B, N
    view: torch.Tensor  # [N, 3] float32, surface -> eye
    image: Optional[Tuple[int, int, int]] = None  # (views, height, width), row-major
    duv: Optional[torch.Tensor] = None  # [N, 4] float32 du/dx, dv/dx, du/dy, dv/dy per pixel
    pos: Optional[torch.Tensor] = None  # [N, 3] float32 scene position of the surface point

    @property
    def count(self) -> int:
        return int(self.uv.shape[0])

    def slice(self, a: int, b: int) -> "GBuffer":
        return GBuffer(self.uv[a:b], self.tbn[a:b], self.view[a:b], None,
                       None if self.duv is None else self.duv[a:b],
                       None if self.pos is None else self.pos[a:b])

    def to(self, device) -> "GBuffer":
        return GBuffer(self.uv.to(device), self.tbn.to(device), self.view.to(device), self.image,
                       None if self.duv is None else self.duv.to(device),
                       None if self.pos is None else self.pos.to(device))


def screen_derivatives(uv: torch.Tensor, views: int, height: int, width: int) -> torch.Tensor:
    """UV screen derivatives of row-major images as a rasteriser's pixel quads
    give them: central differences of the stored coordinates along x and y
    (one-sided at the image border), in binary64, stored as float32 [N, 4]
    (du/dx, dv/dx, du/dy, dv/dy)."""
    g = uv.to(torch.float64).reshape(views, height, width, 2)
    dx = torch.empty_like(g)
    dy = torch.empty_like(g)
    if width > 1:
        dx[:, :, 1:-1] = 0.5 * (g[:, :, 2:] - g[:, :, :-2])
        dx[:, :, 0] = g[:, :, 1] - g[:, :, 0]
        dx[:, :, -1] = g[:, :, -1] - g[:, :, -2]
    else:
        dx.zero_()
    if height > 1:
        dy[:, 1:-1] = 0.5 * (g[:, 2:] - g[:, :-2])
        dy[:, 0] = g[:, 1] - g[:, 0]
        dy[:, -1] = g[:, -1] - g[:, -2]
    else:
        dy.zero_()
    return torch.cat([dx, dy], dim=-1).reshape(-1, 4).to(torch.float32).contiguous()


def flat_gbuffer(N: int, seed: int, device="cpu", min_elev_deg: float = 5.0) -> GBuffer:
    """C1 fragments: UV i.i.d. U[0,1)^2, identity frame, view uniform on the
    spherical cap z in [sin(min_elev), 1] (uniform in z and azimuth)."""
    i = _arange(N, device)
    uv = torch.stack([uniform(seed, S_UV, 2 * i), uniform(seed, S_UV, 2 * i + 1)], dim=1)
    zmin = math.sin(math.radians(min_elev_deg))
    z = zmin + (1.0 - zmin) * uniform64(seed, S_VIEW, 2 * i)
    phi = 2.0 * math.pi * uniform64(seed, S_VIEW, 2 * i + 1)
    r = torch.sqrt(torch.clamp(1.0 - z * z, min=0.0))
    view = torch.stack([r * torch.cos(phi), r * torch.sin(phi), z], dim=1).to(torch.float32)
    tbn = torch.eye(3, dtype=torch.float32, device=device).expand(N, 3, 3).contiguous()
    return GBuffer(uv.contiguous(), tbn, view.contiguous())


def _camera(seed: int, v: int):
    c = uniform64(seed, S_CAMERA, torch.arange(v * 8, v * 8 + 8, dtype=torch.int64))
    h = 1.0 + 4.0 * float(c[0])
    x, y = 8.0 * float(c[1]), 8.0 * float(c[2])
    yaw = 2.0 * math.pi * float(c[3])
    pitch = math.radians(-90.0 + 50.0 * float(c[4]))
    return h, x, y, yaw, pitch


def _rays(h, x, y, yaw, pitch, width, height, device, fov_deg=60.0):
    f = torch.tensor([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw),
                      math.sin(pitch)], dtype=torch.float64, device=device)
    r = torch.tensor([math.sin(yaw), -math.cos(yaw), 0.0], dtype=torch.float64, device=device)
    up = torch.linalg.cross(r, f, dim=0)
    t = math.tan(math.radians(fov_deg) / 2.0)
    aspect = width / height
    px = (2.0 * (torch.arange(width, dtype=torch.float64, device=device) + 0.5) / width - 1.0)
    py = (1.0 - 2.0 * (torch.arange(height, dtype=torch.float64, device=device) + 0.5) / height)
    d = (f[None, None, :] + (px[None, :, None] * t * aspect) * r[None, None, :]
         + (py[:, None, None] * t) * up[None, None, :])
    eye = torch.tensor([x, y, h], dtype=torch.float64, device=device)
    return eye, d.reshape(-1, 3)


def plane_gbuffer(views: int, width: int, height: int, seed: int, device="cpu",
                  normal_sigma_deg: float = 10.0, uv_scale: float = 1.0 / 8.0) -> GBuffer:
    """Perspective views (60 degree vertical FOV, rays through pixel centres)
    of the plane z = 0 with UV = (x, y) / 8.  Camera height U[1,5], position
    U[0,8)^2, yaw U[0, 2 pi), pitch U[-90, -40] degrees, so every pixel hits
    the plane.  Per-pixel normals are tilted by two N(0, sigma) angles."""
    npx = width * height
    uvs, tbns, viewsl, poss = [], [], [], []
    sig = math.radians(normal_sigma_deg)
    for v in range(views):
        h, x, y, yaw, pitch = _camera(seed, v)
        eye, d = _rays(h, x, y, yaw, pitch, width, height, device)
        lam = -h / d[:, 2]
        P = eye[None, :] + lam[:, None] * d
        uv = (P[:, :2] * uv_scale).to(torch.float32)
        vw = -d / torch.linalg.vector_norm(d, dim=1, keepdim=True)
        a, b = normal_pair(seed, S_NORMAL, npx, device, offset=v * npx)
        Nv = torch.stack([torch.tan(a * sig), torch.tan(b * sig), torch.ones_like(a)], dim=1)
        Nv = Nv / torch.linalg.vector_norm(Nv, dim=1, keepdim=True)
        tbn = _frame_from_normal(Nv).to(torch.float32)
        uvs.append(uv)
        tbns.append(tbn)
        viewsl.append(vw.to(torch.float32))
        poss.append(P.to(torch.float32))
        del eye, d, lam, P, Nv
    uv_all = torch.cat(uvs).contiguous()
    return GBuffer(uv_all, torch.cat(tbns).contiguous(), torch.cat(viewsl).contiguous(),
                   (views, height, width), screen_derivatives(uv_all, views, height, width),
                   torch.cat(poss).contiguous())


# --- gradient noise height field (C5) -----------------------------------------

def _lattice_grad(ix: torch.Tensor, iy: torch.Tensor, seed: int):
    # one random unit gradient per integer lattice point (period 4096)
    key = (ix & 4095) * 4096 + (iy & 4095)
    ang = 2.0 * math.pi * uniform64(seed, S_NOISE, key)
    return torch.cos(ang), torch.sin(ang)


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _dfade(t):
    return 30.0 * t * t * (t * (t - 2.0) + 1.0)


def gradient_noise(x: torch.Tensor, y: torch.Tensor, seed: int):
    """Single-octave 2-D gradient noise on the unit lattice with the quintic
    fade 6t^5 - 15t^4 + 10t^3 (Perlin, 2002), and its analytic gradient."""
    x0 = torch.floor(x)
    y0 = torch.floor(y)
    fx, fy = x - x0, y - y0
    ix, iy = x0.to(torch.int64), y0.to(torch.int64)
    vals, grads = [], []
    for dx in (0, 1):
        for dy in (0, 1):
            gx, gy = _lattice_grad(ix + dx, iy + dy, seed)
            rx, ry = fx - dx, fy - dy
            vals.append(gx * rx + gy * ry)
            grads.append((gx, gy))
    u, v = _fade(fx), _fade(fy)
    du, dv = _dfade(fx), _dfade(fy)
    n00, n01, n10, n11 = vals  # (dx,dy) = (0,0),(0,1),(1,0),(1,1)
    nx0 = n00 + u * (n10 - n00)
    nx1 = n01 + u * (n11 - n01)
    val = nx0 + v * (nx1 - nx0)
    (g00x, g00y), (g01x, g01y), (g10x, g10y), (g11x, g11y) = grads
    dnx0_dx = g00x + u * (g10x - g00x) + du * (n10 - n00)
    dnx1_dx = g01x + u * (g11x - g01x) + du * (n11 - n01)
    dnx0_dy = g00y + u * (g10y - g00y)
    dnx1_dy = g01y + u * (g11y - g01y)
    dval_dx = dnx0_dx + v * (dnx1_dx - dnx0_dx)
    dval_dy = dnx0_dy + v * (dnx1_dy - dnx0_dy) + dv * (nx1 - nx0)
    return val, dval_dx, dval_dy


def heightfield_gbuffer(views: int, width: int, height: int, seed: int, device="cpu",
                        amplitude: float = 0.1, uv_scale: float = 1.0 / 8.0,
                        rows_per_chunk: int = 270) -> GBuffer:
    """Perspective views of the height field z = amplitude * noise(x, y).  Each
    ray is bracketed between the planes z = +amplitude and z = -amplitude and
    the crossing of z - h(x, y) is refined by 24 bisection steps.  The frame
    follows the analytic surface gradient."""
    N_all = views * width * height
    uv = torch.empty((N_all, 2), dtype=torch.float32, device=device)
    tbn = torch.empty((N_all, 3, 3), dtype=torch.float32, device=device)
    vw = torch.empty((N_all, 3), dtype=torch.float32, device=device)
    pos = torch.empty((N_all, 3), dtype=torch.float32, device=device)
    for v in range(views):
        h, x, y, yaw, pitch = _camera(seed, v)
        eye, d_all = _rays(h, x, y, yaw, pitch, width, height, device)
        for r0 in range(0, height, rows_per_chunk):
            r1 = min(height, r0 + rows_per_chunk)
            d = d_all[r0 * width:r1 * width]
            t_lo = (h - amplitude) / (-d[:, 2])
            t_hi = (h + amplitude) / (-d[:, 2])
            for _ in range(24):
                tm = 0.5 * (t_lo + t_hi)
                P = eye[None, :] + tm[:, None] * d
                val, _, _ = gradient_noise(P[:, 0], P[:, 1], seed)
                above = P[:, 2] > amplitude * val
                t_lo = torch.where(above, tm, t_lo)
                t_hi = torch.where(above, t_hi, tm)
            tm = 0.5 * (t_lo + t_hi)
            P = eye[None, :] + tm[:, None] * d
            _, hx, hy = gradient_noise(P[:, 0], P[:, 1], seed)
            Nv = torch.stack([-amplitude * hx, -amplitude * hy, torch.ones_like(hx)], dim=1)
            Nv = Nv / torch.linalg.vector_norm(Nv, dim=1, keepdim=True)
            a = v * width * height + r0 * width
            b = v * width * height + r1 * width
            uv[a:b] = (P[:, :2] * uv_scale).to(torch.float32)
            tbn[a:b] = _frame_from_normal(Nv).to(torch.float32)
            vw[a:b] = (-d / torch.linalg.vector_norm(d, dim=1, keepdim=True)).to(torch.float32)
            pos[a:b] = P.to(torch.float32)
        del d_all
    return GBuffer(uv, tbn, vw, (views, height, width),
                   screen_derivatives(uv, views, height, width), pos)


# --- shadow scenes ----------------------------------------------------------------

PLANE_EXTENT = 8.0  # the plane generators map scene (x, y) to UV = (x, y) / 8


def shadow_balls(K: int, seed: int, extent: float = PLANE_EXTENT, zlim=(0.6, 2.0),
                 rlim=(0.15, 0.5)) -> torch.Tensor:
    """K balls [K, 4] float32 (centre x, y, z, radius) over the plane tile
    [0, extent)^2: centres uniform in the tile at heights U[zlim], radii
    U[rlim] (each ball clears the plane)."""
    idx = torch.arange(4 * K, dtype=torch.int64).reshape(K, 4)
    u = uniform64(seed, S_BALLS, idx)
    z = zlim[0] + (zlim[1] - zlim[0]) * u[:, 2]
    r = rlim[0] + (rlim[1] - rlim[0]) * u[:, 3]
    r = torch.minimum(r, 0.9 * z)
    return torch.stack([extent * u[:, 0], extent * u[:, 1], z, r], 1).to(torch.float32)


def bucket_origins(W: int, H: int, extent: float = PLANE_EXTENT, device="cpu") -> torch.Tensor:
    """Scene points of the buckets of a W x H matrix laid over the plane tile
    [0, extent)^2 (UV = (x, y) / extent): the bucket centres, [H, W, 3]."""
    x = (torch.arange(W, dtype=torch.float64, device=device) + 0.5) * (extent / W)
    y = (torch.arange(H, dtype=torch.float64, device=device) + 0.5) * (extent / H)
    o = torch.zeros((H, W, 3), dtype=torch.float64, device=device)
    o[..., 0] = x[None, :]
    o[..., 1] = y[:, None]
    return o.to(torch.float32)


def spiral_cap(axis, half_angle: float, k: int) -> torch.Tensor:
    """k unit directions [k, 3] float64 uniform in solid angle over the cap of
    the given half-angle (radians) around axis, on a golden-angle spiral."""
    i = torch.arange(k, dtype=torch.float64) + 0.5
    cz = 1.0 - i / k * (1.0 - math.cos(half_angle))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    sz = torch.sqrt(torch.clamp(1.0 - cz * cz, min=0.0))
    loc = torch.stack([sz * torch.cos(phi), sz * torch.sin(phi), cz], 1)
    a = torch.tensor(axis, dtype=torch.float64)
    a = a / torch.linalg.vector_norm(a)
    ref = torch.tensor([1.0, 0.0, 0.0] if abs(float(a[0])) < 0.9 else [0.0, 1.0, 0.0],
                       dtype=torch.float64)
    t = torch.linalg.cross(a, ref, dim=0)
    t = t / torch.linalg.vector_norm(t)
    b = torch.linalg.cross(a, t, dim=0)
    return loc @ torch.stack([t, b, a])


def sun_light(k: int, elevation_deg: float = 55.0, azimuth_deg: float = 30.0,
              radius_deg: float = 2.0) -> torch.Tensor:
    """Directions [k, 3] float32 toward a sun disc of the given angular radius."""
    el, az = math.radians(elevation_deg), math.radians(azimuth_deg)
    axis = [math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)]
    return spiral_cap(axis, math.radians(radius_deg), k).to(torch.float32)


def lamp_light(k: int, centre=(4.0, 4.0, 3.0), radius: float = 0.25) -> torch.Tensor:
    """Points [k, 3] float32 on a spherical lamp (the full sphere, uniform by
    area), centre and radius in scene units."""
    d = spiral_cap([0.0, 0.0, 1.0], math.pi, k)
    return (torch.tensor(centre, dtype=torch.float64) + radius * d).to(torch.float32)


def grad_out(N: int, C: int, seed: int, device="cpu") -> torch.Tensor:
    """Upstream gradients, i.i.d. N(0, 1), float32 [N, C]."""
    total = N * C
    half = (total + 1) // 2
    a, b = normal_pair(seed, S_GRAD, half, device)
    return torch.cat([a, b])[:total].to(torch.float32).reshape(N, C)


# ---------------------------------------------------------------------------
# workload table
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    W: int
    H: int
    n: int
    C: int
    views: int
    width: int
    height: int
    seed: int
    kind: str  # "flat", "plane", "heightfield"
    texture: str  # "iid", "smooth"

    @property
    def fragments(self) -> int:
        return self.views * self.width * self.height

    def make_texture(self, device="cpu", seed=None) -> torch.Tensor:
        s = self.seed if seed is None else seed
        if self.texture == "iid":
            return iid_texture(self.W, self.H, self.n, self.C, s, device)
        return smooth_texture(self.W, self.H, self.n, self.C, s, device)

    def make_gbuffer(self, device="cpu") -> GBuffer:
        if self.kind == "flat":
            return flat_gbuffer(self.fragments, self.seed, device)
        if self.kind == "plane":
            return plane_gbuffer(self.views, self.width, self.height, self.seed, device)
        return heightfield_gbuffer(self.views, self.width, self.height, self.seed, device)


WORKLOADS = {
    "c1": Workload("c1_64x64x8x8_rgba_256x256", 64, 64, 8, 4, 1, 256, 256, 1, "flat", "iid"),
    "c2": Workload("c2_1024x1024x16x16_rgba_1920x1080", 1024, 1024, 16, 4, 1, 1920, 1080, 2,
                   "plane", "smooth"),
    "c3": Workload("c3_512x512x16x16_rgba_64x1024x1024", 512, 512, 16, 4, 64, 1024, 1024, 3,
                   "plane", "smooth"),
    "c4": Workload("c4_256x256x8x8_rgb_16x512x512", 256, 256, 8, 3, 16, 512, 512, 4,
                   "plane", "smooth"),
    "c5": Workload("c5_2048x2048x16x16_rgba_8x3840x2160", 2048, 2048, 16, 4, 8, 3840, 2160, 5,
                   "heightfield", "smooth"),
}

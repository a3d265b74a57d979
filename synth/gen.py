"""Clip specification, rendering and the named synthetic workloads."""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

try:
    import scipy.fft as _fft
except Exception:  # pragma: no cover
    _fft = None

# Sampling classes of a shot (same codes as the engine's shot records).
PROG, TFF, BFF, PULLDOWN = 1, 2, 3, 4

# Source-frame index (within a 4-frame group A B C D) of the upper and lower
# field at each position of the 3:2 pulldown unit:
# (Au,Al) (Bu,Bl) (Bu,Cl) (Cu,Dl) (Du,Dl)  -> positions 2 and 3 are mixed.
_PD_UPPER = (0, 1, 1, 2, 3)
_PD_LOWER = (0, 1, 2, 3, 3)


def _pow2_at_least(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


def texture(rng: np.random.Generator, size: int, sigma: float, lo: int, hi: int) -> np.ndarray:
    """size x size toroidal texture: U[0,1) blurred by a periodic Gaussian of
    std `sigma` px, mapped linearly min->lo, max->hi, rounded half up."""
    u = rng.random((size, size), dtype=np.float32)
    f = np.fft.fftfreq(size).astype(np.float32)
    g = np.exp(-2.0 * (math.pi ** 2) * (sigma ** 2) * (f[:, None] ** 2 + f[None, : size // 2 + 1] ** 2))
    if _fft is not None:
        spec = _fft.rfft2(u, workers=8)
        b = _fft.irfft2(spec * g, s=(size, size), workers=8)
    else:
        b = np.fft.irfft2(np.fft.rfft2(u) * g, s=(size, size))
    mn, mx = float(b.min()), float(b.max())
    scale = (hi - lo) / max(mx - mn, 1e-12)
    t = np.floor((b - mn) * scale + lo + 0.5)
    return np.clip(t, lo, hi).astype(np.int32)


@dataclasses.dataclass
class Rect:
    w: int
    h: int
    pos: Tuple[int, int]       # (x, y) at the shot's first frame
    vel: Tuple[int, int]       # px per frame
    tex_seed: int


@dataclasses.dataclass
class ShotSpec:
    length: int                          # frames that belong to the shot
    sampling: int = PROG                 # PROG / TFF / BFF / PULLDOWN
    pan: Optional[List[Tuple[int, int]]] = None  # per-frame (vx, vy); len >= length + 8
    pan_const: Tuple[int, int] = (0, 0)
    offset0: Tuple[int, int] = (0, 0)
    tex_seed: int = 0
    rects: List[Rect] = dataclasses.field(default_factory=list)
    flicker: Optional[Tuple[float, float, float]] = None   # amplitude, Hz, phase
    noise_sigma: float = 0.0
    pd_phase0: int = 0                   # cadence position of the shot's first frame

    def velocity(self, k: int) -> Tuple[int, int]:
        if self.pan is not None:
            return self.pan[min(k, len(self.pan) - 1)]
        return self.pan_const


@dataclasses.dataclass
class ClipSpec:
    W: int
    H: int
    bits: int = 8
    fps: float = 25.0
    lo: int = 16
    hi: int = 235
    tex_sigma: float = 4.0
    rect_sigma: float = 2.0
    shots: List[ShotSpec] = dataclasses.field(default_factory=list)
    transitions: List[int] = dataclasses.field(default_factory=list)  # K per boundary (1 = hardcut)
    flashes: List[int] = dataclasses.field(default_factory=list)
    seed: int = 0
    noise_seed: int = 0
    name: str = ""

    @property
    def T(self) -> int:
        n = sum(s.length for s in self.shots)
        n += sum(k - 1 for k in self.transitions)
        return n

    def layout(self):
        """Per shot: first and last frame; per boundary: (last_old, first_new, K)."""
        firsts, lasts, bounds = [], [], []
        f = 0
        for i, s in enumerate(self.shots):
            firsts.append(f)
            lasts.append(f + s.length - 1)
            f += s.length
            if i < len(self.transitions):
                k = self.transitions[i]
                bounds.append((f - 1, f - 1 + k, k))
                f += k - 1
        return firsts, lasts, bounds

    def truth(self) -> Dict:
        firsts, lasts, bounds = self.layout()
        shots = []
        for i, s in enumerate(self.shots):
            k = 0 if i == 0 else self.transitions[i - 1]
            shots.append({"first": firsts[i], "last": lasts[i], "in_k": k,
                          "in_boundary": 0 if i == 0 else (1 if k == 1 else 2),
                          "sampling": s.sampling,
                          "pulldown_phase": (-s.pd_phase0 + 2) % 5 if s.sampling == PULLDOWN else -1,
                          "pan": s.pan_const})
        return {"T": self.T, "shots": shots, "boundaries": bounds, "flashes": list(self.flashes)}


class Renderer:
    """Renders frame t of a ClipSpec (uint8 for 8-bit, uint16 otherwise)."""

    def __init__(self, spec: ClipSpec):
        self.spec = spec
        self.P = _pow2_at_least(2 * max(spec.W, spec.H))
        self._tex: Dict[int, np.ndarray] = {}
        self._rtex: Dict[Tuple[int, int, int], np.ndarray] = {}
        self.firsts, self.lasts, self.bounds = spec.layout()
        self.T = spec.T
        self._shot_of = np.zeros(self.T, np.int32)
        self._trans: Dict[int, Tuple[int, int, int]] = {}
        for i in range(len(spec.shots)):
            self._shot_of[self.firsts[i]:self.lasts[i] + 1] = i
        for i, (last_old, first_new, k) in enumerate(self.bounds):
            for f in range(last_old + 1, first_new):
                self._trans[f] = (i, f - last_old, k)
                self._shot_of[f] = -1
        self._flash = set(spec.flashes)
        self._yy = np.arange(spec.H)[:, None]
        self._xx = np.arange(spec.W)[None, :]

    def _bg(self, i: int) -> np.ndarray:
        if i not in self._tex:
            s = self.spec
            rng = np.random.Generator(np.random.PCG64(s.shots[i].tex_seed))
            self._tex[i] = texture(rng, self.P, s.tex_sigma, s.lo, s.hi)
        return self._tex[i]

    def _rect_tex(self, r: Rect) -> np.ndarray:
        key = (r.tex_seed, r.w, r.h)
        if key not in self._rtex:
            s = self.spec
            size = _pow2_at_least(max(r.w, r.h))
            rng = np.random.Generator(np.random.PCG64(r.tex_seed))
            self._rtex[key] = texture(rng, size, s.rect_sigma, s.lo, s.hi)
        return self._rtex[key]

    def _offset(self, shot: ShotSpec, tau2: int) -> Tuple[int, int]:
        """Background offset at time tau = tau2 / 2 frames after the shot's start
        (for half times the frame's velocity must be even)."""
        ox, oy = shot.offset0
        k = tau2 // 2
        for j in range(k):
            vx, vy = shot.velocity(j)
            ox -= vx
            oy -= vy
        if tau2 % 2:
            vx, vy = shot.velocity(k)
            ox -= vx // 2
            oy -= vy // 2
        return ox, oy

    def scene(self, i: int, tau2: int) -> np.ndarray:
        """Shot i's scene at time tau2/2 frames after its first frame (int32)."""
        s = self.spec
        shot = s.shots[i]
        P = self.P
        ox, oy = self._offset(shot, tau2)
        tex = self._bg(i)
        rows = (self._yy[:, 0] + oy) % P
        cols = (self._xx[0, :] + ox) % P
        img = tex[np.ix_(rows, cols)]
        for r in shot.rects:
            rt = self._rect_tex(r)
            rs = rt.shape[0]
            px = r.pos[0] + (r.vel[0] * tau2) // 2
            py = r.pos[1] + (r.vel[1] * tau2) // 2
            ys = (py + np.arange(r.h)) % s.H
            xs = (px + np.arange(r.w)) % s.W
            img[np.ix_(ys, xs)] = rt[np.ix_(np.arange(r.h) % rs, np.arange(r.w) % rs)]
        return img

    def _shot_frame(self, i: int, k: int) -> np.ndarray:
        """Frame k of shot i (k may run past the shot into a dissolve)."""
        shot = self.spec.shots[i]
        if shot.sampling == PROG:
            return self.scene(i, 2 * k)
        if shot.sampling in (TFF, BFF):
            early = self.scene(i, 2 * k)
            late = self.scene(i, 2 * k + 1)
            out = early.copy()
            if shot.sampling == TFF:
                out[1::2] = late[1::2]      # upper (even rows) first
            else:
                out[0::2] = late[0::2]      # lower (odd rows) first
            return out
        # 3:2 pulldown: source frames run at 4/5 of the video frame rate; the
        # source scene advances one velocity step per source frame.
        pos = (k + shot.pd_phase0) % 5
        unit = (k + shot.pd_phase0) // 5
        su = 4 * unit + _PD_UPPER[pos]
        sl = 4 * unit + _PD_LOWER[pos]
        base = 4 * (shot.pd_phase0 // 5) + _PD_UPPER[shot.pd_phase0 % 5]
        up = self.scene(i, 2 * (su - base))
        out = up.copy()
        if sl != su:
            lo = self.scene(i, 2 * (sl - base))
            out[1::2] = lo[1::2]
        return out

    def frame(self, t: int, rng_noise: Optional[np.random.Generator] = None) -> np.ndarray:
        s = self.spec
        i = int(self._shot_of[t])
        if i >= 0:
            img = self._shot_frame(i, t - self.firsts[i])
            shot = s.shots[i]
        else:
            b, k, K = self._trans[t]
            a_img = self._shot_frame(b, t - self.firsts[b])
            b_img = self._shot_frame(b + 1, t - self.firsts[b + 1])
            img = ((K - k) * a_img + k * b_img + K // 2) // K
            shot = s.shots[b + 1]
        img = img.astype(np.int32)
        if shot.flicker is not None:
            amp, hz, ph = shot.flicker
            img += int(np.rint(amp * math.sin(2 * math.pi * hz * t / s.fps + ph)))
        if t in self._flash:
            img += 60 if s.bits == 8 else 240
        if shot.noise_sigma > 0:
            rng = rng_noise if rng_noise is not None else np.random.Generator(
                np.random.PCG64([s.noise_seed, t]))
            n = rng.standard_normal((s.H, s.W), dtype=np.float32)
            img += np.rint(n * np.float32(shot.noise_sigma)).astype(np.int32)
        maxv = (1 << s.bits) - 1
        np.clip(img, 0, maxv, out=img)
        return img.astype(np.uint8 if s.bits == 8 else np.uint16)


def render(spec: ClipSpec, frames=None) -> np.ndarray:
    """Render the given frame indices (default: all) into one array [n, H, W]."""
    r = Renderer(spec)
    idx = list(range(spec.T)) if frames is None else list(frames)
    out = np.empty((len(idx), spec.H, spec.W), np.uint8 if spec.bits == 8 else np.uint16)
    for j, t in enumerate(idx):
        out[j] = r.frame(t)
    return out


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def _working_level(W: int, wmax: int = 512) -> int:
    L = 0
    while W > wmax:
        W //= 2
        L += 1
    return L


def make_c1(seed: int = 1, T: int = 64, W: int = 320, H: int = 180) -> ClipSpec:
    """Single progressive 320x180 clip, 25 fps: smooth-noise background
    (sigma 4 px, 16..235) moved by iid integer motion in [-4, 4] per frame,
    a hardcut to a fresh background at frame T/2, Gaussian noise sigma 2."""
    ss = np.random.SeedSequence(seed)
    s_tex, s_mot, s_off, s_noise = ss.spawn(4)
    mrng = np.random.Generator(np.random.PCG64(s_mot))
    orng = np.random.Generator(np.random.PCG64(s_off))
    cut = T // 2
    shots = []
    for i, n in enumerate((cut, T - cut)):
        pan = [tuple(int(v) for v in mrng.integers(-4, 5, size=2)) for _ in range(n + 16)]
        shots.append(ShotSpec(length=n, sampling=PROG, pan=pan,
                              offset0=tuple(int(v) for v in orng.integers(0, 4096, size=2)),
                              tex_seed=int(s_tex.generate_state(1)[0]) + i, noise_sigma=2.0))
    return ClipSpec(W=W, H=H, bits=8, fps=25.0, shots=shots, transitions=[1],
                    tex_sigma=4.0, rect_sigma=2.0, seed=seed,
                    noise_seed=int(s_noise.generate_state(1)[0]), name="c1")


def _shot_lengths(rng, T, lo, hi, k_dis, p_dis):
    lens, trans = [], []
    used = 0
    while True:
        n = int(rng.integers(lo, hi + 1))
        k = k_dis if rng.random() < p_dis else 1
        if used + n + (k - 1) + lo > T:
            lens.append(T - used)
            break
        lens.append(n)
        trans.append(k)
        used += n + k - 1
    return lens, trans


def _even_pan(rng, lim, min_inf):
    while True:
        v = rng.integers(-lim // 2, lim // 2 + 1, size=2) * 2
        if max(abs(int(v[0])), abs(int(v[1]))) >= min_inf:
            return (int(v[0]), int(v[1]))


def _make_general(seed: int, T: int, W: int, H: int, bits: int, fps: float,
                  sampling_probs: Dict[int, float], pan_lim: int, min_inter_pan: int,
                  k_dis: int, p_dis: float, shot_lo: int, shot_hi: int,
                  noise: Tuple[float, float], flash_p: float, flicker_p: float,
                  lo: int, hi: int, tex_sigma0: float, rect_sigma0: float,
                  rect_count: Tuple[int, int], rect_vel: int, name: str) -> ClipSpec:
    ss = np.random.SeedSequence(seed)
    s_layout, s_shot, s_flash, s_noise = ss.spawn(4)
    rng = np.random.Generator(np.random.PCG64(s_layout))
    srng = np.random.Generator(np.random.PCG64(s_shot))
    L = _working_level(W)
    lens, trans = _shot_lengths(rng, T, shot_lo, shot_hi, k_dis, p_dis)
    classes = list(sampling_probs.keys())
    probs = np.array([sampling_probs[c] for c in classes], np.float64)
    probs /= probs.sum()
    shots = []
    for i, n in enumerate(lens):
        samp = int(classes[int(srng.choice(len(classes), p=probs))])
        if samp == PROG:
            v = tuple(int(x) for x in srng.integers(-pan_lim, pan_lim + 1, size=2))
        else:
            v = _even_pan(srng, pan_lim, min_inter_pan)
        rects = []
        for _ in range(int(srng.integers(rect_count[0], rect_count[1] + 1))):
            rw = int(srng.integers(W // 16, W // 4 + 1))
            rh = int(srng.integers(H // 16, H // 4 + 1))
            rv = tuple(int(x) for x in srng.integers(-rect_vel // 2, rect_vel // 2 + 1, size=2) * 2)
            rects.append(Rect(w=rw, h=rh,
                              pos=(int(srng.integers(0, W)), int(srng.integers(0, H))),
                              vel=rv, tex_seed=int(srng.integers(1, 2 ** 62))))
        flick = None
        if srng.random() < flicker_p:
            flick = (10.0 if bits == 8 else 40.0, float(srng.uniform(2.0, 5.0)),
                     float(srng.uniform(0, 2 * math.pi)))
        shots.append(ShotSpec(length=n, sampling=samp, pan_const=v,
                              offset0=(int(srng.integers(0, 1 << 16)), int(srng.integers(0, 1 << 16))),
                              tex_seed=int(srng.integers(1, 2 ** 62)), rects=rects, flicker=flick,
                              noise_sigma=float(srng.uniform(noise[0], noise[1])),
                              pd_phase0=int(srng.integers(0, 5))))
    spec = ClipSpec(W=W, H=H, bits=bits, fps=fps, lo=lo, hi=hi,
                    tex_sigma=tex_sigma0 * (1 << L), rect_sigma=rect_sigma0 * (1 << L),
                    shots=shots, transitions=trans, seed=seed,
                    noise_seed=int(s_noise.generate_state(1)[0]), name=name)
    # one-frame flashes, never within 2 frames of a boundary or of the clip ends
    frng = np.random.Generator(np.random.PCG64(s_flash))
    firsts, lasts, bounds = spec.layout()
    near = set()
    for last_old, first_new, _ in bounds:
        for f in range(last_old - 2, first_new + 3):
            near.add(f)
    Tn = spec.T
    spec.flashes = [t for t in range(3, Tn - 3) if t not in near and frng.random() < flash_p]
    return spec


def make_c2(seed: int = 2, T: int = 1500, W: int = 2048, H: int = 1080, k_dis: int = 8) -> ClipSpec:
    """2K plain-method clip: 2048x1080 8-bit, 25 fps; smooth-noise backgrounds
    plus 3-6 moving textured rectangles; pans up to 32 px/frame; hardcuts
    (p 0.7) or k_dis-frame linear dissolves (p 0.3) every 100-300 frames;
    progressive / TFF / BFF / 3:2 pulldown shots; one-frame +60 flashes;
    +-10 flicker at 2-5 Hz on 30% of shots; noise sigma 3-8."""
    sc = W / 2048.0   # motion scales with the frame size (the working level is ~512 wide)
    return _make_general(seed, T, W, H, 8, 25.0, {PROG: 0.4, TFF: 0.2, BFF: 0.2, PULLDOWN: 0.2},
                         pan_lim=max(2, int(round(32 * sc))), min_inter_pan=max(2, int(round(8 * sc))) // 2 * 2,
                         k_dis=k_dis, p_dis=0.3,
                         shot_lo=100, shot_hi=300, noise=(3.0, 8.0), flash_p=0.01, flicker_p=0.3,
                         lo=16, hi=235, tex_sigma0=4.0, rect_sigma0=2.0, rect_count=(3, 6),
                         rect_vel=max(2, int(round(16 * sc))), name="c2")


# The batched mix: (W, H, interlaced, fps)
MIX_FORMATS = [
    (720, 576, True, 25.0),
    (1280, 720, False, 50.0),
    (1920, 1080, False, 25.0),
    (1920, 1080, True, 25.0),
    (2048, 1080, False, 24.0),
    (3840, 2160, False, 25.0),
]


def make_mix_clip(i: int, seed: int = 3, T: Optional[int] = None, k_dis: int = 8) -> ClipSpec:
    """Clip i of the uneven batched mix: format i mod 6, length U{200..3000}
    (or T), the 2K generator scaled to the format."""
    W, H, inter, fps = MIX_FORMATS[i % len(MIX_FORMATS)]
    rng = np.random.Generator(np.random.PCG64([seed, i]))
    n = int(rng.integers(200, 3001)) if T is None else T
    probs = {TFF: 0.4, BFF: 0.4, PROG: 0.2} if inter else {PROG: 1.0}
    scale = W / 2048.0
    return _make_general(seed * 100003 + i, n, W, H, 8, fps, probs,
                         pan_lim=max(8, int(32 * scale) // 2 * 2), min_inter_pan=8, k_dis=k_dis,
                         p_dis=0.3, shot_lo=min(100, max(20, n // 3)), shot_hi=min(300, max(40, n)),
                         noise=(3.0, 8.0), flash_p=0.01, flicker_p=0.3, lo=16, hi=235,
                         tex_sigma0=4.0, rect_sigma0=2.0, rect_count=(3, 6), rect_vel=16,
                         name=f"mix{i}")


def make_c5(seed: int = 5, T: int = 45000, W: int = 3840, H: int = 2160) -> ClipSpec:
    """Stress: 4K 10-bit (uint16) 50i, low contrast 64..192 (10-bit units),
    pans up to 64 px/frame (even, >= 16), noise sigma 12, flashes p 1/25 at
    +240, hardcuts every 100-300 frames, no dissolves."""
    return _make_general(seed, T, W, H, 10, 25.0, {TFF: 0.5, BFF: 0.5},
                         pan_lim=64, min_inter_pan=16, k_dis=1, p_dis=0.0,
                         shot_lo=100, shot_hi=300, noise=(12.0, 12.0), flash_p=1.0 / 25,
                         flicker_p=0.0, lo=64, hi=192, tex_sigma0=4.0, rect_sigma0=2.0,
                         rect_count=(3, 6), rect_vel=16, name="c5")

"""Frames of a ClipSpec rendered with torch on a device.

The throughput runs need clips at their full lengths (hundreds to tens of
thousands of frames, up to 3840x2160), which the numpy renderer takes minutes
to produce.  This renderer follows the same recipe step for step (toroidal
background crop at the shot's offset, opaque textured rectangles, interlaced
and 3:2 pulldown field merges, K-frame linear dissolves, flicker, flash,
Gaussian noise, clip) with torch tensors, so a clip renders in a fraction of
a second per hundred frames on a GPU.

Random numbers: with host_noise the texture noise and the per-frame Gaussian
noise come from the same numpy generators as Renderer (then frames equal
Renderer's except where the two FFT implementations round a texture value to
a different integer, a few pixels in 10^4 by at most 1).  Without it they
come from torch's generator on the device, seeded by the same per-shot and
per-frame seeds: the clip has the same structure and statistics but other
pixel values.  Like the rest of this package it holds none of the measure
engine's arithmetic.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

from .gen import PROG, TFF, BFF, _PD_LOWER, _PD_UPPER, ClipSpec, Renderer, _pow2_at_least

_MASK63 = (1 << 63) - 1


class DeviceRenderer:
    """Renders frames t0 .. t0+n-1 of a ClipSpec into a torch tensor."""

    def __init__(self, spec: ClipSpec, device="cuda:0", host_noise: bool = False, max_pixels: int = 1 << 25):
        import torch
        self.torch = torch
        self.spec = spec
        self.dev = torch.device(device)
        self.host_noise = host_noise
        self.max_pixels = max_pixels
        self.lay = Renderer(spec)          # shot layout, offsets and transitions (no pixels)
        self.P = _pow2_at_least(2 * max(spec.W, spec.H))
        self._tex: Dict[int, object] = {}
        self._rtex: Dict[Tuple[int, int, int], object] = {}
        self._yy = torch.arange(spec.H, device=self.dev)
        self._xx = torch.arange(spec.W, device=self.dev)
        self.dtype = torch.uint8 if spec.bits == 8 else torch.int16

    # -- textures ---------------------------------------------------------
    def _texture(self, seed: int, size: int, sigma: float, lo: int, hi: int):
        torch = self.torch
        if self.host_noise:
            rng = np.random.Generator(np.random.PCG64(seed))
            u = torch.from_numpy(rng.random((size, size), dtype=np.float32)).to(self.dev)
        else:
            g = torch.Generator(device=self.dev)
            g.manual_seed(int(seed) & _MASK63)
            u = torch.rand((size, size), generator=g, device=self.dev, dtype=torch.float32)
        f = torch.fft.fftfreq(size, device=self.dev, dtype=torch.float32)
        gk = torch.exp(-2.0 * (math.pi ** 2) * (sigma ** 2) * (f[:, None] ** 2 + f[None, : size // 2 + 1] ** 2))
        b = torch.fft.irfft2(torch.fft.rfft2(u) * gk, s=(size, size))
        del u
        mn, mx = float(b.min()), float(b.max())
        scale = (hi - lo) / max(mx - mn, 1e-12)
        t = torch.floor((b - mn) * scale + lo + 0.5)
        return torch.clamp(t, lo, hi).to(torch.int32)

    def _bg(self, i: int):
        if i not in self._tex:
            if len(self._tex) >= 3:                      # frames are rendered in order: keep the latest shots
                del self._tex[min(self._tex)]
            s = self.spec
            self._tex[i] = self._texture(s.shots[i].tex_seed, self.P, s.tex_sigma, s.lo, s.hi)
        return self._tex[i]

    def _rect_tex(self, r):
        key = (r.tex_seed, r.w, r.h)
        if key not in self._rtex:
            if len(self._rtex) >= 32:
                self._rtex.clear()
            s = self.spec
            size = _pow2_at_least(max(r.w, r.h))
            rt = self._texture(r.tex_seed, size, s.rect_sigma, s.lo, s.hi)
            ar = self.torch.arange(r.h, device=self.dev) % size
            ac = self.torch.arange(r.w, device=self.dev) % size
            self._rtex[key] = rt[ar[:, None], ac[None, :]]
        return self._rtex[key]

    # -- composition ------------------------------------------------------
    def _scenes(self, i: int, tau2: List[int]):
        """Shot i's scene at each time tau2/2 after its first frame: [n, H, W] int32."""
        torch = self.torch
        s = self.spec
        shot = s.shots[i]
        P = self.P
        if shot.pan is None:                 # constant pan: the offset in closed form
            vx, vy = shot.pan_const
            k = np.array(tau2, np.int64) // 2
            odd = np.array(tau2, np.int64) % 2
            off = np.stack([shot.offset0[0] - k * vx - odd * (vx // 2),
                            shot.offset0[1] - k * vy - odd * (vy // 2)], 1)
        else:
            off = np.array([self.lay._offset(shot, t) for t in tau2], np.int64)
        ox = torch.from_numpy(off[:, 0]).to(self.dev)
        oy = torch.from_numpy(off[:, 1]).to(self.dev)
        rows = torch.remainder(self._yy[None, :] + oy[:, None], P)
        cols = torch.remainder(self._xx[None, :] + ox[:, None], P)
        img = self._bg(i)[rows[:, :, None], cols[:, None, :]]
        n = len(tau2)
        tt = torch.tensor(tau2, device=self.dev, dtype=torch.int64)
        nn = torch.arange(n, device=self.dev)[:, None, None]
        for r in shot.rects:
            vals = self._rect_tex(r)
            px = torch.div(r.vel[0] * tt, 2, rounding_mode="floor") + r.pos[0]
            py = torch.div(r.vel[1] * tt, 2, rounding_mode="floor") + r.pos[1]
            ys = torch.remainder(py[:, None] + torch.arange(r.h, device=self.dev)[None, :], s.H)
            xs = torch.remainder(px[:, None] + torch.arange(r.w, device=self.dev)[None, :], s.W)
            img[nn, ys[:, :, None], xs[:, None, :]] = vals[None].expand(n, r.h, r.w)
        return img

    def _shot_frames(self, i: int, ks: List[int]):
        """Frames k of shot i (k may run past the shot into a dissolve)."""
        shot = self.spec.shots[i]
        if shot.sampling == PROG:
            return self._scenes(i, [2 * k for k in ks])
        if shot.sampling in (TFF, BFF):
            early = self._scenes(i, [2 * k for k in ks])
            late = self._scenes(i, [2 * k + 1 for k in ks])
            if shot.sampling == TFF:
                early[:, 1::2] = late[:, 1::2]
            else:
                early[:, 0::2] = late[:, 0::2]
            return early
        base = 4 * (shot.pd_phase0 // 5) + _PD_UPPER[shot.pd_phase0 % 5]
        su, sl = [], []
        for k in ks:
            pos = (k + shot.pd_phase0) % 5
            unit = (k + shot.pd_phase0) // 5
            su.append(4 * unit + _PD_UPPER[pos])
            sl.append(4 * unit + _PD_LOWER[pos])
        up = self._scenes(i, [2 * (u - base) for u in su])
        mixed = [j for j in range(len(ks)) if sl[j] != su[j]]
        if mixed:
            lo = self._scenes(i, [2 * (sl[j] - base) for j in mixed])
            idx = self.torch.tensor(mixed, device=self.dev)
            sel = up[idx]
            sel[:, 1::2] = lo[:, 1::2]
            up[idx] = sel
        return up

    def _finish(self, img, ts: List[int], shots: List[int]):
        """Flicker, flash, noise and clip of frames ts (their shots' effects)."""
        torch = self.torch
        s = self.spec
        add = np.zeros(len(ts), np.int64)
        for j, (t, si) in enumerate(zip(ts, shots)):
            shot = s.shots[si]
            if shot.flicker is not None:
                amp, hz, ph = shot.flicker
                add[j] += int(np.rint(amp * math.sin(2 * math.pi * hz * t / s.fps + ph)))
            if t in self.lay._flash:
                add[j] += 60 if s.bits == 8 else 240
        if add.any():
            img += torch.from_numpy(add).to(self.dev, torch.int32)[:, None, None]
        for j, (t, si) in enumerate(zip(ts, shots)):
            sigma = s.shots[si].noise_sigma
            if sigma <= 0:
                continue
            if self.host_noise:
                rng = np.random.Generator(np.random.PCG64([s.noise_seed, t]))
                nz = torch.from_numpy(rng.standard_normal((s.H, s.W), dtype=np.float32)).to(self.dev)
            else:
                g = torch.Generator(device=self.dev)
                g.manual_seed((int(s.noise_seed) * 1000003 + t) & _MASK63)
                nz = torch.randn((s.H, s.W), generator=g, device=self.dev, dtype=torch.float32)
            img[j] += torch.round(nz * np.float32(sigma)).to(torch.int32)
        maxv = (1 << s.bits) - 1
        return torch.clamp(img, 0, maxv).to(self.dtype)

    def render_into(self, out, t0: int = 0):
        """Fill out[j] with frame t0 + j (out: [n, H, W] uint8, or int16 holding
        10-bit samples, on the renderer's device)."""
        s = self.spec
        n = out.shape[0]
        assert t0 >= 0 and t0 + n <= self.lay.T and tuple(out.shape[1:]) == (s.H, s.W)
        step = max(1, self.max_pixels // (s.H * s.W))
        t = t0
        while t < t0 + n:
            i = int(self.lay._shot_of[t])
            if i < 0:                                       # a dissolve frame
                b, k, K = self.lay._trans[t]
                a_img = self._shot_frames(b, [t - self.lay.firsts[b]])
                b_img = self._shot_frames(b + 1, [t - self.lay.firsts[b + 1]])
                img = self.torch.div((K - k) * a_img + k * b_img + K // 2, K, rounding_mode="floor")
                out[t - t0] = self._finish(img, [t], [b + 1])[0]
                t += 1
                continue
            hi = min(t0 + n, self.lay.lasts[i] + 1, t + step)
            ts = list(range(t, hi))
            img = self._shot_frames(i, [u - self.lay.firsts[i] for u in ts])
            out[t - t0:hi - t0] = self._finish(img, ts, [i] * len(ts))
            t = hi
        return out

    def frames(self, t0: int, n: int):
        out = self.torch.empty((n, self.spec.H, self.spec.W), dtype=self.dtype, device=self.dev)
        return self.render_into(out, t0)

"""Planetary ephemerides from SPK files (Sect. 3.2: perturber positions are
read from precomputed SPICE kernels), ingested into the library's table.

An SPK file is a NAIF DAF container: a 1024-byte file record, a linked
list of summary records (each followed by a name record) and the segment
data, all addressed in 8-byte words counted from 1.  Each summary holds
the segment's start and end epoch (TDB seconds past J2000) and six
integers: target, centre, frame, data type, first and last word.  Types 2
(Chebyshev position) and 3 (Chebyshev position and velocity) store
records of [mid, radius, coefficients...] of equal length, closed by the
four words [init, intlen, rsize, n].

`load_spk` reads those segments, chains every requested body to the
solar-system barycentre (NAIF id 0) through the segments' centres, and
resamples the barycentric positions into uniform segments of
`seg_days` days and a fixed degree (Chebyshev-Gauss interpolation), the
layout `kete_ephem_t` takes.  Units become au and TDB days past J2000.

Frames (App. A.1): the library integrates in the ecliptic J2000 frame,
while planetary kernels such as DE440 store the equatorial J2000 frame
(NAIF frame 1, taken as the ICRF).  Segments in frame 1 are rotated to the
ecliptic by the J2000 obliquity about the common x axis (the equinox);
segments in frame 17 (ECLIPJ2000) are taken as they are; any other frame
is refused.  Only little-endian files are read.  `write_spk` writes
type-2 and type-3 files (used to make test fixtures).
"""
from __future__ import annotations

import dataclasses
import struct
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import synth

AU_KM = synth.AU_KM
DAY_S = 86400.0
_REC = 1024

FRAME_J2000 = 1            # NAIF: equatorial J2000 (ICRF)
FRAME_ECLIPJ2000 = 17      # NAIF: ecliptic J2000
OBLIQUITY_J2000 = np.radians(84381.448 / 3600.0)    # IAU mean obliquity at J2000, rad


def equatorial_to_ecliptic(x: np.ndarray) -> np.ndarray:
    """Vectors [..., 3] of the equatorial J2000 frame in the ecliptic J2000
    frame: a rotation by the obliquity about the x axis (the equinox)."""
    c, s = np.cos(OBLIQUITY_J2000), np.sin(OBLIQUITY_J2000)
    x = np.asarray(x, float)
    return np.stack([x[..., 0], c * x[..., 1] + s * x[..., 2], -s * x[..., 1] + c * x[..., 2]], -1)


@dataclasses.dataclass
class Segment:
    target: int
    center: int
    frame: int
    dtype: int
    et0: float
    et1: float
    init: float
    intlen: float
    n_comp: int              # 3 (type 2) or 6 (type 3)
    coef: np.ndarray         # [n_rec][n_comp][deg+1], km
    mid: np.ndarray          # [n_rec] seconds
    radius: np.ndarray       # [n_rec] seconds

    def position(self, et: np.ndarray) -> np.ndarray:
        """Position [..., 3] in km of target relative to centre at et (s)."""
        et = np.asarray(et, float)
        k = np.clip(np.floor((et - self.init) / self.intlen).astype(np.int64), 0, self.mid.size - 1)
        x = (et - self.mid[k]) / self.radius[k]
        c = self.coef[k][..., :3, :]                        # [..., 3, deg+1]
        # Chebyshev series by the three-term recurrence
        t_prev = np.ones_like(x)
        out = c[..., 0] * t_prev[..., None]
        if c.shape[-1] > 1:
            t_cur = x
            out = out + c[..., 1] * t_cur[..., None]
            for j in range(2, c.shape[-1]):
                t_prev, t_cur = t_cur, 2.0 * x * t_cur - t_prev
                out = out + c[..., j] * t_cur[..., None]
        return out

    def position_ecliptic(self, et: np.ndarray) -> np.ndarray:
        """position() in the ecliptic J2000 frame (km)."""
        p = self.position(et)
        if self.frame == FRAME_ECLIPJ2000:
            return p
        if self.frame == FRAME_J2000:
            return equatorial_to_ecliptic(p)
        raise ValueError(f"segment of body {self.target}: frame {self.frame} is neither J2000 (1) nor "
                         f"ECLIPJ2000 (17)")


def read_segments(path: str) -> List[Segment]:
    """Every type 2 or type 3 segment of an SPK file."""
    data = np.memmap(path, dtype=np.uint8, mode="r")
    head = bytes(data[:_REC])
    if head[:7] != b"DAF/SPK":
        raise ValueError(f"{path}: not a DAF/SPK file")
    if head[88:96] != b"LTL-IEEE":
        raise ValueError(f"{path}: only little-endian (LTL-IEEE) files are read")
    nd, ni = struct.unpack("<ii", head[8:16])
    fward = struct.unpack("<i", head[76:80])[0]
    if nd != 2 or ni != 6:
        raise ValueError(f"{path}: unexpected summary format ND={nd} NI={ni}")
    words = np.frombuffer(data, dtype="<f8")
    ss = nd + (ni + 1) // 2
    segs: List[Segment] = []
    rec = fward
    seen = set()
    while rec > 0 and rec not in seen:
        seen.add(rec)
        base = (rec - 1) * (_REC // 8)
        nxt, _prev, nsum = words[base:base + 3]
        for i in range(int(nsum)):
            w = base + 3 + i * ss
            et0, et1 = words[w], words[w + 1]
            ints = np.frombuffer(words[w + 2:w + 2 + (ni + 1) // 2].tobytes(), dtype="<i4")[:ni]
            target, center, frame, dtype, a0, a1 = (int(v) for v in ints)
            if dtype not in (2, 3):
                continue
            init, intlen, rsize, n = words[a1 - 4:a1]
            rsize, n = int(rsize), int(n)
            n_comp = 3 if dtype == 2 else 6
            deg1 = (rsize - 2) // n_comp
            recs = np.array(words[a0 - 1:a0 - 1 + rsize * n]).reshape(n, rsize)
            segs.append(Segment(target, center, frame, dtype, float(et0), float(et1), float(init), float(intlen),
                                n_comp, recs[:, 2:2 + n_comp * deg1].reshape(n, n_comp, deg1).copy(),
                                recs[:, 0].copy(), recs[:, 1].copy()))
        rec = int(nxt)
    return segs


def _covering(segs: Sequence[Segment], target: int, et: np.ndarray) -> Segment:
    cand = [s for s in segs if s.target == target and s.et0 <= et.min() and s.et1 >= et.max()]
    if not cand:
        raise ValueError(f"no segment for body {target} covers [{et.min():.1f}, {et.max():.1f}] s")
    return cand[-1]          # later segments take precedence, as in SPICE


def barycentric(segs: Sequence[Segment], target: int, et: np.ndarray) -> np.ndarray:
    """Position [..., 3] in km of `target` relative to the solar-system
    barycentre in the ecliptic J2000 frame, chaining segments through their
    centres (each rotated from its own frame)."""
    et = np.asarray(et, float)
    pos = np.zeros(et.shape + (3,))
    body, hops = target, 0
    while body != 0:
        s = _covering(segs, body, et)
        pos = pos + s.position_ecliptic(et)
        body, hops = s.center, hops + 1
        if hops > 16:
            raise ValueError(f"centre chain of body {target} does not reach the barycentre")
    return pos


def load_spk(paths: Sequence[str], bodies: Sequence[int], gm: Sequence[float], t_start: float, t_end: float,
             seg_days: float = synth.SEG_DAYS, degree: int = synth.CHEB_DEGREE,
             gr_bodies: Sequence[int] = (10, 5, 399), names: Optional[List[str]] = None) -> synth.Ephemeris:
    """Barycentric positions of `bodies` (NAIF ids, body 0 of the table
    first: the Sun, 10) from the SPK files, resampled over
    [t_start, t_end] (TDB days past J2000) into uniform segments."""
    segs: List[Segment] = []
    for p in paths:
        segs += read_segments(p)
    n_seg = int(np.ceil((t_end - t_start) / seg_days - 1e-12))
    x = synth.cheb_fit_nodes(degree)
    W = synth.cheb_fit_matrix(degree)
    t0 = t_start + seg_days * np.arange(n_seg)
    tn = t0[:, None] + 0.5 * seg_days * (x[None, :] + 1.0)            # [seg, node] days
    coef = np.empty((len(bodies), n_seg, 3, degree + 1))
    for b, naif in enumerate(bodies):
        pos = barycentric(segs, naif, tn * DAY_S) / AU_KM               # [seg, node, 3] au
        coef[b] = np.einsum("kj,sjc->sck", W, pos)
    flags = np.array([1 if n in gr_bodies else 0 for n in bodies], np.uint32)
    return synth.Ephemeris(np.ascontiguousarray(coef), np.asarray(gm, float), flags, float(t_start),
                           float(seg_days), names or [str(n) for n in bodies])


def write_spk(path: str, segments: Sequence[dict]) -> None:
    """Write a little-endian SPK file.  Each segment dict holds target,
    center, frame (the frame its numbers are in: 1 equatorial J2000, 17
    ecliptic J2000; required), init (s), intlen (s) and coef: [n_rec][3][deg+1]
    km for type 2, or [n_rec][6][deg+1] (positions in km, then velocities in
    km/s) for type 3; record i covers [init + i intlen, init + (i+1) intlen]."""
    nd, ni = 2, 6
    ss = nd + (ni + 1) // 2
    if len(segments) > (_REC // 8 - 3) // ss:
        raise ValueError("too many segments for one summary record")
    words: List[float] = []
    summaries = []
    addr = 3 * (_REC // 8) + 1                  # data start after file, summary and name records
    for sg in segments:
        c = np.asarray(sg["coef"], float)
        n, n_comp, deg1 = c.shape
        if n_comp not in (3, 6):
            raise ValueError("coef must hold 3 (type 2) or 6 (type 3) components")
        rsize = 2 + n_comp * deg1
        init, intlen = float(sg["init"]), float(sg["intlen"])
        a0 = addr + len(words)
        for i in range(n):
            words += [init + (i + 0.5) * intlen, 0.5 * intlen] + c[i].reshape(-1).tolist()
        words += [init, intlen, float(rsize), float(n)]
        a1 = addr + len(words) - 1
        summaries.append((init, init + n * intlen, sg["target"], sg["center"], int(sg["frame"]),
                          2 if n_comp == 3 else 3, a0, a1))
    free = addr + len(words)
    fr = bytearray(_REC)
    fr[0:8] = b"DAF/SPK "
    fr[8:16] = struct.pack("<ii", nd, ni)
    fr[16:76] = b"synthetic test ephemeris".ljust(60)
    fr[76:88] = struct.pack("<iii", 2, 2, free)
    fr[88:96] = b"LTL-IEEE"
    sr = np.zeros(_REC // 8)
    sr[:3] = [0.0, 0.0, float(len(summaries))]
    for i, (e0, e1, tg, ce, fm, ty, a0, a1) in enumerate(summaries):
        w = 3 + i * ss
        sr[w:w + 2] = [e0, e1]
        sr[w + 2:w + ss] = np.frombuffer(struct.pack("<6i", tg, ce, fm, ty, a0, a1), dtype="<f8")
    nr = bytearray(_REC)
    with open(path, "wb") as f:
        f.write(bytes(fr))
        f.write(sr.astype("<f8").tobytes())
        f.write(bytes(nr))
        f.write(np.asarray(words, "<f8").tobytes())

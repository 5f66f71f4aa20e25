"""Zel'dovich-displaced particle grids (seeded, synthetic).

The paper measures on cosmological N-body snapshots (its Results section);
those are not available here, so every input is drawn from a Gaussian random
displacement field instead.  Recipe (all in float64 numpy, C order, x slowest):

1. w = standard_normal((Np, Np, Np)) from ``numpy.random.default_rng(seed)``.
2. W = rfftn(w); integer wavevectors k_j from fftfreq(Np) * Np.
3. psi_hat_j = i k_j / |k|^2 * W, so the displacement power spectrum falls as
   k^-2.  The k = 0 mode and every mode on a Nyquist plane are zeroed.
4. psi_j = irfftn(psi_hat_j), scaled so that the rms over all three
   components equals ``rms`` Lagrangian spacings.
5. x = ((q + psi) / Np) mod 1 with q the lattice index; cast to float32, and
   a value that rounds to 1.0f becomes 0.0f.

Optional clumps contract space around seeded centres (monotone radial map, so
they add no extra shell crossing).  The module only produces positions.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "zeldovich_positions",
    "apply_clumps",
    "lattice_positions",
    "jittered_lattice_positions",
    "batched_box_specs",
    "workload",
    "WORKLOADS",
]


def _finish(x: np.ndarray) -> np.ndarray:
    """Wrap into [0,1), cast to float32, map 1.0f to 0.0f."""
    x = np.mod(x, 1.0)
    xf = x.astype(np.float32)
    xf[xf >= np.float32(1.0)] = np.float32(0.0)
    return np.ascontiguousarray(xf)


def lattice_positions(np_: int) -> np.ndarray:
    """Undisplaced lattice: particle (i,j,k) at (i,j,k)/Np.  float32 [Np,Np,Np,3]."""
    q = np.indices((np_, np_, np_), dtype=np.float64)
    x = np.moveaxis(q, 0, -1) / np_
    return _finish(x)


def _displacement(np_: int, rms: float, seed: int, spectrum: str = "displacement",
                  rms_mode: str = "component") -> np.ndarray:
    """Displacement field psi in Lagrangian spacings, float64 [Np,Np,Np,3]."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((np_, np_, np_))
    W = np.fft.rfftn(w)
    del w
    kx = np.fft.fftfreq(np_) * np_
    kz = np.fft.rfftfreq(np_) * np_
    KX = kx[:, None, None]
    KY = kx[None, :, None]
    KZ = kz[None, None, :]
    k2 = KX * KX + KY * KY + KZ * KZ
    k2[0, 0, 0] = 1.0
    if spectrum == "displacement":
        amp = 1.0 / k2                      # |psi_hat|^2 ~ k^2 / k^4 = k^-2
    elif spectrum == "density":
        amp = 1.0 / (k2 * np.sqrt(k2))      # |delta_hat|^2 ~ k^-2
    else:
        raise ValueError(spectrum)
    amp[0, 0, 0] = 0.0
    nyq = np_ // 2
    if np_ % 2 == 0:
        amp[np.abs(kx) == nyq, :, :] = 0.0
        amp[:, np.abs(kx) == nyq, :] = 0.0
        amp[:, :, np.abs(kz) == nyq] = 0.0
    psi = np.empty((np_, np_, np_, 3), dtype=np.float64)
    for j, K in enumerate((KX, KY, KZ)):
        psi[..., j] = np.fft.irfftn(1j * K * amp * W, s=(np_, np_, np_), axes=(0, 1, 2))
    del W
    if rms_mode == "component":
        cur = np.sqrt(np.mean(psi * psi))
    elif rms_mode == "vector":
        cur = np.sqrt(np.mean(np.sum(psi * psi, axis=-1)))
    else:
        raise ValueError(rms_mode)
    if cur > 0:
        psi *= rms / cur
    return psi


def zeldovich_positions(np_: int, rms: float, seed: int, spectrum: str = "displacement",
                        rms_mode: str = "component") -> np.ndarray:
    """Periodic unit-box particle positions, float32 [Np,Np,Np,3] (x slowest)."""
    psi = _displacement(np_, rms, seed, spectrum, rms_mode)
    q = np.indices((np_, np_, np_), dtype=np.float64)
    psi += np.moveaxis(q, 0, -1)
    psi /= np_
    return _finish(psi)


def jittered_lattice_positions(np_: int, amplitude: float, seed: int) -> np.ndarray:
    """Lattice plus independent uniform offsets in [-amplitude, amplitude] spacings per axis.

    This is the analytic input the paper uses for its weak-scaling runs
    (offsets of up to one cell width in each direction, Weak Scaling section).
    """
    rng = np.random.default_rng(seed)
    q = np.moveaxis(np.indices((np_, np_, np_), dtype=np.float64), 0, -1)
    off = rng.uniform(-amplitude, amplitude, size=q.shape)
    return _finish((q + off) / np_)


def apply_clumps(pos: np.ndarray, n_centres: int = 100, radius: float = 0.01,
                 compression: float = 10.0, seed: int = 1003, cutoff: float = 0.0625) -> np.ndarray:
    """Contract space around seeded centres: x <- c + d (1 - (1 - s) exp(-|d|^2 / 2R^2)).

    d is the minimum image of x - c and s = compression^(-1/3), so the central
    density rises by ``compression``.  Applied centre by centre, wrapping after
    each.  Particles with |d| >= cutoff are left unchanged (at 6.25 radii the
    displacement is below 1e-9 box).  Candidates come from a binning of the
    current positions (bins no smaller than the cutoff); particles that change
    bin are tracked separately, so every particle within the cutoff is found.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_centres, 3))
    s = compression ** (-1.0 / 3.0)
    x = pos.astype(np.float64).reshape(-1, 3)
    nb = max(3, int(np.floor(1.0 / cutoff)))
    bs = 1.0 / nb

    def bins_of(pts):
        b = np.floor(np.mod(pts, 1.0) / bs).astype(np.int64)
        np.clip(b, 0, nb - 1, out=b)
        return ((b[:, 0] * nb + b[:, 1]) * nb + b[:, 2]).astype(np.uint16)

    key = bins_of(x)
    order = np.argsort(key, kind="stable")
    starts = np.searchsorted(key[order], np.arange(nb ** 3 + 1))
    is_stale = np.zeros(x.shape[0], dtype=bool)
    stale = np.zeros(0, dtype=np.int64)
    for c in centres:
        cb = np.floor(c / bs).astype(np.int64)
        parts = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    bx, by, bz = (cb[0] + dx) % nb, (cb[1] + dy) % nb, (cb[2] + dz) % nb
                    b = (bx * nb + by) * nb + bz
                    parts.append(order[starts[b]:starts[b + 1]])
        cand = np.concatenate(parts)
        cand = np.unique(cand) if nb < 3 else cand
        cand = np.concatenate([cand[~is_stale[cand]], stale])
        d = x[cand] - c
        d -= np.rint(d)
        r2 = np.sum(d * d, axis=1)
        sel = r2 < cutoff * cutoff
        idx = cand[sel]
        f = 1.0 - (1.0 - s) * np.exp(-r2[sel] / (2.0 * radius * radius))
        x[idx] = np.mod(c + d[sel] * f[:, None], 1.0)
        nk = bins_of(x[idx])
        moved = idx[nk != key[idx]]
        if moved.size:
            key[moved] = bins_of(x[moved])
            new = moved[~is_stale[moved]]
            is_stale[new] = True
            stale = np.concatenate([stale, new])
    return _finish(x.reshape(pos.shape))


def batched_box_specs(seed: int = 4, n_boxes: int = 64):
    """Independent boxes of uneven size: list of dicts (np, rms, seed, nc)."""
    rng = np.random.default_rng(seed)
    specs = []
    for b in range(n_boxes):
        np_ = int(rng.choice([16, 32, 64, 128]))
        rms = float(rng.uniform(0.3, 3.0))
        specs.append({"np": np_, "rms": rms, "seed": 4000 + b, "nc": 2 * np_})
    return specs


# Named workloads: particle grid, displacement, seed and deposit target.
WORKLOADS = {
    # 32^3 particles, rms 0.5 spacing -> 64^3 periodic grid (196,608 tets)
    "zel32_g64": {"np": 32, "rms": 0.5, "seed": 1, "nc": 64},
    # 256^3 particles, rms 2.0 spacings -> 512^3 grid (~100.7M tets)
    "zel256_g512": {"np": 256, "rms": 2.0, "seed": 2, "nc": 512},
    # 512^3 particles, rms 3.0 spacings plus 100 clumps -> octree of 16^3 blocks
    "clump512_octree": {"np": 512, "rms": 3.0, "seed": 3, "clumps": 1003,
                        "block": 16, "max_level": 4, "threshold": 1 << 20},
    # 256^3 particles, rms 2.0 spacings -> 64^3 grid (most tets fit 2x2x2 cells)
    "zel256_g64": {"np": 256, "rms": 2.0, "seed": 6, "nc": 64},
    # the same geometry (0.25 cells per spacing) at 64^3 particles -> 16^3 grid
    "zel64_g16": {"np": 64, "rms": 2.0, "seed": 7, "nc": 16},
}

# Seeds of the boxes that supply surrogate training examples (never used for
# evaluation, which takes the workloads' own seeds).
TRAIN_SEED0 = 5000


def uniform_segments(segments, seed: int) -> np.ndarray:
    """Concatenated float32 draws U(-b, b) for segments [(count, b), ...] (initial weights)."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.uniform(-b, b, size=int(n)) for n, b in segments]).astype(
        np.float32)


def workload(name: str, seed: int | None = None) -> tuple[np.ndarray, dict]:
    """Positions and parameters of a named workload (seed may be overridden)."""
    p = dict(WORKLOADS[name])
    if seed is not None:
        p["seed"] = seed
    pos = zeldovich_positions(p["np"], p["rms"], p["seed"])
    if "clumps" in p:
        pos = apply_clumps(pos, seed=p["clumps"])
    return pos, p

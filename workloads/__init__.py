"""Seeded synthetic user drops for the near-field XL-MIMO Gram workloads.

This module only draws inputs: array descriptions, per-drop antenna counts,
per-drop user counts and user positions in metres.  It holds none of the
method's arithmetic (no channel, Gram, closed form or rate), so both the FP64
oracle and the HIP path can take their inputs from it without sharing any code
that computes a result.

Geometry conventions (paper, Sec. II-A, antenna scheme): the array lies in the
x = 0 plane, centred at the origin; a ULA runs along the y axis.  A user at
(x, y, z) sees the array from the x > 0 half-space.  Angles are measured from
broadside (+x): x = r cos(theta), y = r sin(theta).

Every generator takes an explicit ``numpy.random.Generator``; ``rng_for``
builds the PCG64 stream used by the named workloads, seeded with
``SEED_BASE + workload index``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

SEED_BASE = 20250318
SPEED_OF_LIGHT = 299_792_458.0

GEOM_ULA = 0
GEOM_UPA = 1
AMP_FREESPACE = 0
AMP_PNUSW = 1


@dataclasses.dataclass(frozen=True)
class ArraySpec:
    """Receive array: ULA (n_z == 1) along y, or UPA in the y-z plane."""

    geometry: int
    n_y: int
    n_z: int
    spacing: float
    wavelength: float
    amp_model: int = AMP_FREESPACE
    beta0: float = 1.0

    @property
    def n_elems(self) -> int:
        return int(self.n_y) * int(self.n_z)

    def with_n(self, n: int) -> "ArraySpec":
        """Same ULA with a different element count."""
        assert self.geometry == GEOM_ULA
        return dataclasses.replace(self, n_y=int(n), n_z=1)


@dataclasses.dataclass
class Drops:
    """A batch of Monte-Carlo drops, possibly uneven in N and K.

    n_elems[d]  antennas used by drop d (ULA: elements along y)
    n_users[d]  users in drop d
    user_off    prefix sums of n_users, length n_drops + 1
    pos         [total_users, 3] float64 user coordinates (x, y, z) in metres
    """

    n_elems: np.ndarray
    n_users: np.ndarray
    user_off: np.ndarray
    pos: np.ndarray

    @property
    def n_drops(self) -> int:
        return int(self.n_users.shape[0])

    @property
    def total_users(self) -> int:
        return int(self.user_off[-1])

    def gram_off(self) -> np.ndarray:
        """Prefix sums of K_d^2 (offsets of each drop's K x K block)."""
        k = self.n_users.astype(np.int64)
        return np.concatenate([[0], np.cumsum(k * k)]).astype(np.int64)

    def users_of(self, d: int) -> np.ndarray:
        return self.pos[self.user_off[d]:self.user_off[d + 1]]

    def subset(self, idx: Sequence[int]) -> "Drops":
        idx = list(idx)
        pos = np.concatenate([self.users_of(d) for d in idx]) if idx else np.zeros((0, 3))
        k = self.n_users[idx].astype(np.int32)
        off = np.concatenate([[0], np.cumsum(k.astype(np.int64))]).astype(np.int64)
        return Drops(self.n_elems[idx].astype(np.int64), k, off, np.ascontiguousarray(pos))

    def with_n(self, n: int) -> "Drops":
        return Drops(np.full(self.n_drops, int(n), np.int64), self.n_users.copy(),
                     self.user_off.copy(), self.pos.copy())


def rng_for(workload_index: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([SEED_BASE + int(workload_index), int(stream)]))


def _pack(n_elems, n_users, pos) -> Drops:
    n_users = np.asarray(n_users, np.int32)
    off = np.concatenate([[0], np.cumsum(n_users.astype(np.int64))]).astype(np.int64)
    return Drops(np.asarray(n_elems, np.int64), n_users, off, np.ascontiguousarray(pos, np.float64))


def polar_drops(rng, n_drops: int, k: int, n_elems: int, r_range, theta_deg, log_r=False) -> Drops:
    """K users per drop, distance uniform (or log-uniform) and angle uniform."""
    r_lo, r_hi = r_range
    if log_r:
        r = np.exp(rng.uniform(math.log(r_lo), math.log(r_hi), size=(n_drops, k)))
    else:
        r = rng.uniform(r_lo, r_hi, size=(n_drops, k))
    th = np.deg2rad(rng.uniform(theta_deg[0], theta_deg[1], size=(n_drops, k)))
    pos = np.stack([r * np.cos(th), r * np.sin(th), np.zeros_like(r)], axis=-1).reshape(-1, 3)
    return _pack(np.full(n_drops, n_elems), np.full(n_drops, k), pos)


def uneven_drops(rng, n_drops: int, n_range, k_range, r_range, theta_deg) -> Drops:
    """Per drop: K ~ U{k_lo..k_hi}, N ~ U{n_lo..n_hi}, then log-uniform r and uniform angle."""
    ks = rng.integers(k_range[0], k_range[1] + 1, size=n_drops)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=n_drops)
    tot = int(ks.sum())
    r = np.exp(rng.uniform(math.log(r_range[0]), math.log(r_range[1]), size=tot))
    th = np.deg2rad(rng.uniform(theta_deg[0], theta_deg[1], size=tot))
    pos = np.stack([r * np.cos(th), r * np.sin(th), np.zeros_like(r)], axis=-1)
    return _pack(ns, ks, pos)


def cone_drops(rng, n_drops: int, k: int, n_elems: int, r_range, az_deg, el_deg) -> Drops:
    """Users in a 3-D cone: r, azimuth and elevation independent and uniform."""
    r = rng.uniform(r_range[0], r_range[1], size=(n_drops, k))
    az = np.deg2rad(rng.uniform(az_deg[0], az_deg[1], size=(n_drops, k)))
    el = np.deg2rad(rng.uniform(el_deg[0], el_deg[1], size=(n_drops, k)))
    pos = np.stack([r * np.cos(el) * np.cos(az), r * np.cos(el) * np.sin(az), r * np.sin(el)],
                   axis=-1).reshape(-1, 3)
    return _pack(np.full(n_drops, n_elems), np.full(n_drops, k), pos)


def rect_drops(rng, n_drops: int, k: int, n_elems: int, x_range, y_range) -> Drops:
    """Users uniform in a rectangle beside the array (the paper's Sec. IV/V scenes)."""
    x = rng.uniform(x_range[0], x_range[1], size=(n_drops, k))
    y = rng.uniform(y_range[0], y_range[1], size=(n_drops, k))
    pos = np.stack([x, y, np.zeros_like(x)], axis=-1).reshape(-1, 3)
    return _pack(np.full(n_drops, n_elems), np.full(n_drops, k), pos)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

LAMBDA_28GHZ = 10.71e-3           # as written for the 28 GHz workloads
LAMBDA_100GHZ_UPA = 3.0e-3        # as written for the 100 GHz UPA workload
LAMBDA_100GHZ = SPEED_OF_LIGHT / 100e9   # the paper's 100 GHz scenes

SWEEP_N = (256, 1024, 4096, 16384, 65536, 262144)


def ula(n: int, wavelength: float, amp_model: int = AMP_FREESPACE, spacing: Optional[float] = None) -> ArraySpec:
    return ArraySpec(GEOM_ULA, int(n), 1, wavelength / 2 if spacing is None else spacing,
                     wavelength, amp_model)


def plain_fp64(n_drops: int = 1000):
    """ULA N=256 at 28 GHz, K=4, r ~ U[5,50] m, angle ~ U[-60,60] deg, SNR 10 dB."""
    arr = ula(256, LAMBDA_28GHZ)
    drops = polar_drops(rng_for(0), n_drops, 4, 256, (5.0, 50.0), (-60.0, 60.0))
    return arr, drops, dict(snr_db=(10.0,), ref_distance=27.5)


def sweep(n_drops: int = 10_000, n_list=SWEEP_N):
    """Sweep of ULA sizes, K=16, same user distribution as plain_fp64, SNR {0,10,20} dB."""
    arr = ula(n_list[-1], LAMBDA_28GHZ)
    drops = polar_drops(rng_for(1), n_drops, 16, n_list[-1], (5.0, 50.0), (-60.0, 60.0))
    return arr, drops, dict(snr_db=(0.0, 10.0, 20.0), ref_distance=27.5, n_list=tuple(n_list))


def uneven(n_drops: int = 4096):
    """Uneven batch: N ~ U{1024..262144}, K ~ U{2..32}, r log-uniform [2,100] m, angle U[-75,75]."""
    arr = ula(262144, LAMBDA_28GHZ)
    drops = uneven_drops(rng_for(2), n_drops, (1024, 262144), (2, 32), (2.0, 100.0), (-75.0, 75.0))
    # Mean distance of a log-uniform law on [2,100] m: (100-2)/ln(50) = 25.05 m.
    return arr, drops, dict(snr_db=(10.0,), ref_distance=(100.0 - 2.0) / math.log(50.0))


def upa(n_drops: int = 2000):
    """UPA 512x512 at 100 GHz (lambda = 3.0 mm, half-wavelength spacing), K=64 users in a cone."""
    arr = ArraySpec(GEOM_UPA, 512, 512, LAMBDA_100GHZ_UPA / 2, LAMBDA_100GHZ_UPA, AMP_FREESPACE)
    drops = cone_drops(rng_for(3), n_drops, 64, 512 * 512, (3.0, 30.0), (-60.0, 60.0), (-60.0, 60.0))
    return arr, drops, dict(snr_db=(10.0,), ref_distance=16.5)


def learned_pairs(n_pairs: int, stream: int = 0, n_list=SWEEP_N):
    """Two-user drops over the sweep's user law and N set (training/inference pairs for the MLP)."""
    rng = rng_for(4, stream)
    ns = rng.choice(np.asarray(n_list, np.int64), size=n_pairs)
    r = rng.uniform(5.0, 50.0, size=(n_pairs, 2))
    th = np.deg2rad(rng.uniform(-60.0, 60.0, size=(n_pairs, 2)))
    pos = np.stack([r * np.cos(th), r * np.sin(th), np.zeros_like(r)], axis=-1).reshape(-1, 3)
    return ula(n_list[-1], LAMBDA_28GHZ), _pack(ns, np.full(n_pairs, 2), pos)


def paper_sec4(n_drops: int = 100, n: int = 65536):
    """Paper Sec. IV scene: 100 GHz, x ~ U[1,10] m, y ~ U[-7.5,7.5] m, K=100, PNUSW, t=0.9."""
    arr = ula(n, LAMBDA_100GHZ, AMP_PNUSW)
    drops = rect_drops(rng_for(10), n_drops, 100, n, (1.0, 10.0), (-7.5, 7.5))
    return arr, drops, dict(t=0.9, snr_db=(0.0, 200.0))


def paper_sec5(n_drops: int = 100, n: int = 16384):
    """Paper Sec. V scene: as Sec. IV but x ~ U(1,2) m and K=10; received SNR limit 33 dB at (1.5 m, 0)."""
    arr = ula(n, LAMBDA_100GHZ, AMP_PNUSW)
    drops = rect_drops(rng_for(11), n_drops, 10, n, (1.0, 2.0), (-7.5, 7.5))
    return arr, drops, dict(t=0.9, rx_snr_limit_db=33.0, ref_point=(1.5, 0.0))


def learned_calibration(n_drops: int = 4000, n_list=SWEEP_N):
    """Held-out drops of the sweep's law (K=16, the same positions at every N) on which the
    learned correction's fallback thresholds are calibrated; disjoint from the training
    drops and from the sweep workload's drops."""
    arr = ula(n_list[-1], LAMBDA_28GHZ)
    drops = polar_drops(rng_for(4, 7), n_drops, 16, n_list[-1], (5.0, 50.0), (-60.0, 60.0))
    return arr, drops, dict(snr_db=(0.0, 10.0, 20.0), ref_distance=27.5, n_list=tuple(n_list))


def learned_drops(n_drops: int, stream: int = 0, k: int = 16, n_list=SWEEP_N):
    """Drops of K users over the sweep's user law, N drawn per drop from the sweep's N set
    (training and evaluation pairs of the learned correction: K(K-1)/2 pairs per drop)."""
    rng = rng_for(4, stream)
    ns = rng.choice(np.asarray(n_list, np.int64), size=n_drops)
    r = rng.uniform(5.0, 50.0, size=(n_drops, k))
    th = np.deg2rad(rng.uniform(-60.0, 60.0, size=(n_drops, k)))
    pos = np.stack([r * np.cos(th), r * np.sin(th), np.zeros_like(r)], axis=-1).reshape(-1, 3)
    return ula(n_list[-1], LAMBDA_28GHZ), _pack(ns, np.full(n_drops, k), pos)

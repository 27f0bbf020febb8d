"""Seeded synthetic traffic tensors with the shapes and structure of the paper's workloads.

The paper evaluates on the Abilene and GEANT traffic matrices (section 5), which are not
available here.  These generators stand in for them with tensors of the same kind:

* mode 1 = origin-destination (OD) pairs, mode 2 = time slots of a day, mode 3 = days
  (the tube); values are non-negative traffic volumes;
* a low-tubal-rank core (the model of section 3.1 assumes the completed tensor is a
  t-product of an n1 x r x n3 and an r x n2 x n3 tensor), scaled per OD pair by
  heavy-tailed log-normal magnitudes, multiplied by a diurnal profile along mode 2 and,
  optionally, a weekly profile along mode 3;
* additive Gaussian noise relative to the RMS of the clean tensor, then clipping at 0;
* a uniformly random observation mask (the "random missing pattern" of section 5);
* initial factors X0 = 0 and Y0 ~ N(0, 1).

Everything here is input data.  The low-rank core is synthesised through numpy's FFT
(rank-r products of the tube-frequency slices, transformed back); neither the oracle nor
the GPU library imports anything from this module except the arrays it returns.

Recipe (draw order fixed; ``rng = numpy.random.default_rng(seed)``):

    Xg ~ N(1, 1)^(n1 x r x n3);  Yg ~ N(1, 1)^(r x n2 x n3)
    L  = core of tubal rank <= r built from Xg, Yg
    L *= lognormal(0, sigma_od)[i]            (per OD pair)
    L *= 1 + 0.3 sin(2 pi j / n2)             (diurnal, mode 2)
    L *= 1 + 0.3 sin(2 pi k / 7)              (weekly, mode 3, when enabled)
    M  = max(L + noise * rms(L) * N(0, 1), 0)
    u  = uniform[0, 1);  Omega = u < p;  held-out = p <= u < p + 0.1
    Y0 ~ N(0, 1) from default_rng(seed + 1);  X0 = 0

Unit-mean factors keep the clipping rare (zero-mean factors would zero about half the
entries and destroy the low-rank structure).
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    """A named synthetic completion problem."""

    name: str
    n1: int            # OD pairs (mode 1)
    n2: int            # time slots per day (mode 2)
    n3: int            # days (mode 3, the tube)
    r: int             # tubal rank of the model
    sigma_od: float    # log-normal sigma of the per-OD magnitudes
    weekly: bool       # multiply a period-7 profile along the tube
    noise: float       # additive noise, relative to RMS of the clean tensor
    p: float           # sampling rate of Omega
    iters: int         # iterations the workload is run for
    mu: float = 1e-2   # ridge weight on W
    rho1: float = 1e-2 # temporal-stability weight (H, mode 1)
    rho2: float = 1e-2 # periodicity weight (K, mode 2)
    seed: int = 0
    holdout: bool = False


WORKLOADS: dict[str, Workload] = {
    # plain method, small: 36 OD x 48 slots x 7 days, tubal rank 3, 30 % sampled
    "od36x48x7_r3": Workload("od36x48x7_r3", 36, 48, 7, 3, 1.0, False, 0.01, 0.30, 50),
    # plain method, 5-minute slots over four weeks, rank 8, at five sampling rates
    **{
        f"od144x288x28_r8_p{int(p * 100)}": Workload(
            f"od144x288x28_r8_p{int(p * 100)}", 144, 288, 28, 8, 1.0, True, 0.02, p, 200)
        for p in (0.1, 0.2, 0.4, 0.6, 0.8)
    },
    # precision workload: 529 OD x 96 fifteen-minute slots x 112 days, rank 16, 40 % sampled
    "od529x96x112_r16": Workload("od529x96x112_r16", 529, 96, 112, 16, 1.5, True, 0.02, 0.40, 200),
    # differentiation workload: 40 % sampled plus 10 % held out
    "od144x288x28_r8_holdout": Workload(
        "od144x288x28_r8_holdout", 144, 288, 28, 8, 1.0, True, 0.02, 0.40, 20, holdout=True),
}


def _low_tubal_rank_core(xg: np.ndarray, yg: np.ndarray) -> np.ndarray:
    """Real n1 x n2 x n3 tensor whose tube-frequency slices are products of xg's and yg's."""
    n3 = xg.shape[2]
    xf = np.fft.rfft(xg, axis=2).transpose(2, 0, 1)      # (bins, n1, r)
    yf = np.fft.rfft(yg, axis=2).transpose(2, 0, 1)      # (bins, r, n2)
    lf = np.matmul(xf, yf).transpose(1, 2, 0)            # (n1, n2, bins)
    return np.fft.irfft(lf, n=n3, axis=2)


def make_inputs(n1: int, n2: int, n3: int, r: int, *, sigma_od: float = 1.0,
                weekly: bool = False, noise: float = 0.01, p: float = 0.3,
                seed: int = 0, holdout: bool = False) -> dict:
    """Draw one synthetic problem.  Returns float32 / uint8 arrays in C order.

    Keys: ``M`` full tensor (n1, n2, n3); ``G`` = M on Omega and 0 elsewhere;
    ``omega`` 0/1 mask; ``holdout`` 0/1 mask of held-out entries (or None);
    ``X0`` (n1, r, n3) zeros; ``Y0`` (r, n2, n3) standard normal.
    """
    if min(n1, n2, n3, r) < 1:
        raise ValueError("all sizes must be >= 1")
    rng = np.random.default_rng(seed)
    xg = rng.normal(1.0, 1.0, size=(n1, r, n3))
    yg = rng.normal(1.0, 1.0, size=(r, n2, n3))
    core = _low_tubal_rank_core(xg, yg)
    od_scale = rng.lognormal(0.0, sigma_od, size=n1)
    core = core * od_scale[:, None, None]
    j = np.arange(n2)
    core = core * (1.0 + 0.3 * np.sin(2.0 * np.pi * j / n2))[None, :, None]
    if weekly:
        k = np.arange(n3)
        core = core * (1.0 + 0.3 * np.sin(2.0 * np.pi * k / 7.0))[None, None, :]
    rms = float(np.sqrt(np.mean(core * core)))
    m = np.maximum(core + noise * rms * rng.normal(0.0, 1.0, size=core.shape), 0.0)
    u = rng.random(size=core.shape)
    omega = u < p
    hold = ((u >= p) & (u < p + 0.1)) if holdout else None

    rng0 = np.random.default_rng(seed + 1)
    y0 = rng0.normal(0.0, 1.0, size=(r, n2, n3))
    x0 = np.zeros((n1, r, n3))

    m32 = np.ascontiguousarray(m, dtype=np.float32)
    g32 = np.where(omega, m32, np.float32(0.0)).astype(np.float32)
    return {
        "M": m32,
        "G": np.ascontiguousarray(g32),
        "omega": np.ascontiguousarray(omega.astype(np.uint8)),
        "holdout": None if hold is None else np.ascontiguousarray(hold.astype(np.uint8)),
        "X0": np.ascontiguousarray(x0, dtype=np.float32),
        "Y0": np.ascontiguousarray(y0, dtype=np.float32),
    }


def make_workload(name_or_workload, **overrides) -> tuple[Workload, dict]:
    """Inputs of a named workload (optionally with fields overridden)."""
    w = WORKLOADS[name_or_workload] if isinstance(name_or_workload, str) else name_or_workload
    if overrides:
        w = replace(w, **overrides)
    data = make_inputs(w.n1, w.n2, w.n3, w.r, sigma_od=w.sigma_od, weekly=w.weekly,
                       noise=w.noise, p=w.p, seed=w.seed, holdout=w.holdout)
    return w, data


def batch_specs(count: int = 64, seed: int = 1) -> list[Workload]:
    """Sizes of a batch of uneven completions: for each completion, in this order,
    n1 from {36, 144, 529}, n2 from {48, 96, 288}, n3 from {7, 28, 112}, r uniform in
    [2, 16] and p uniform in [0.2, 0.6), all drawn from ``default_rng(seed)``; data seed
    1000 + t, log-normal(0, 1) OD scales, diurnal and weekly profiles, 2 % noise, 50
    iterations."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n1 = int(rng.choice([36, 144, 529]))
        n2 = int(rng.choice([48, 96, 288]))
        n3 = int(rng.choice([7, 28, 112]))
        r = int(rng.integers(2, 17))
        p = float(rng.uniform(0.2, 0.6))
        out.append(Workload(f"batch{t}_{n1}x{n2}x{n3}_r{r}", n1, n2, n3, r, 1.0, True, 0.02, p, 50,
                            seed=1000 + t))
    return out


LAYOUTS = {
    # the generator's layout: OD pair x time slot x day (mode 3, the tube, is the day)
    "od_slot_day": "OD pair x slot x day",
    # the paper's model layout t x d x o (section 3.1): slot x day x OD pair
    "slot_day_od": "slot x day x OD pair",
    # the router-pair layout of the paper's experiments (N x N x T): origin x destination x
    # time, with time running over the days' slots in order (T = slots x days)
    "origin_destination_time": "origin x destination x time",
}


def relayout(d: dict, layout: str, r: int, seed: int) -> dict:
    """The same observations in another layout: M, G and the masks permuted (or reshaped),
    and a new start X0 = 0, Y0 ~ N(0, 1) of the new shape from default_rng(seed + 1).  Input
    arrays are (o, t, d) = (OD pair, slot, day); the origin-destination form needs o = N^2."""
    def move(a):
        if a is None:
            return None
        if layout == "od_slot_day":
            return a
        if layout == "slot_day_od":
            return np.ascontiguousarray(np.transpose(a, (1, 2, 0)))
        if layout == "origin_destination_time":
            o, t, dd = a.shape
            n = int(round(np.sqrt(o)))
            if n * n != o:
                raise ValueError("the origin x destination layout needs a square number of OD pairs")
            return np.ascontiguousarray(np.transpose(a, (0, 2, 1)).reshape(n, n, dd * t))
        raise KeyError(layout)
    out = {k: move(d[k]) for k in ("M", "G", "omega", "holdout")}
    n1, n2, n3 = out["M"].shape
    rng0 = np.random.default_rng(seed + 1)
    out["Y0"] = np.ascontiguousarray(rng0.normal(0.0, 1.0, size=(r, n2, n3)), dtype=np.float32)
    out["X0"] = np.zeros((n1, r, n3), dtype=np.float32)
    return out

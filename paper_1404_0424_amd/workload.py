"""Seeded synthetic inputs for massive-MIMO uplink detection and downlink precoding.

This module only *draws* inputs: channels, transmitted bits and symbols, noise.
It holds none of the detection or precoding arithmetic, so both the FP64 oracle
and the GPU path can be fed from it without sharing any of the method's code.

System model (Sec. II): per subcarrier, uplink y = H_u x + n (eq. (1)) with
H_u in C^{B x U}, x drawn from a square Gray-labelled QAM alphabet O with
E|x_i|^2 = E_s, and n ~ CN(0, N0 I).  Downlink symbols t in O^U are precoded.

Array conventions (shared with the C ABI, all row-major, complex128 here):
  H  (n_sc, B, U)   uplink channel H_u per subcarrier
  Y  (n_sc, B, S)   receive vectors of S OFDM symbols as columns
  X  (n_sc, U, S)   transmitted symbols, bits (n_sc, U, S, m)
  T  (n_sc, U, S)   downlink symbols to precode

The paper's channels come from the WINNER-II model, which is not available
here; i.i.d. Rayleigh and Kronecker-correlated Rayleigh channels at the same
antenna counts stand in for it.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 14040424


def rng_for(config: int, index: int = 0) -> np.random.Generator:
    """PCG64 stream for workload ``config`` and frame ``index``."""
    return np.random.default_rng(SEED_BASE + 1000 * config + index)


# --------------------------------------------------------------------------
# channels
# --------------------------------------------------------------------------

def iid_channel(rng: np.random.Generator, n_sc: int, B: int, U: int) -> np.ndarray:
    """i.i.d. CN(0, 1/B) entries, shape (n_sc, B, U)."""
    s = math.sqrt(0.5 / B)
    return (rng.standard_normal((n_sc, B, U)) * s
            + 1j * rng.standard_normal((n_sc, B, U)) * s)


def exp_corr(n: int, rho: float) -> np.ndarray:
    """Exponential correlation matrix [R]_ij = rho^|i-j|."""
    idx = np.arange(n)
    return rho ** np.abs(idx[:, None] - idx[None, :])


def kronecker_channel(rng: np.random.Generator, n_sc: int, B: int, U: int,
                      rho_bs: float, rho_ue: float) -> np.ndarray:
    """Kronecker model H = L_B H_w L_U^T with L L^T = R (Cholesky factors).

    With H_w i.i.d. CN(0, 1/B) this has E[H H^H] proportional to R_B and
    E[H^H H] proportional to R_U; the Cholesky factor gives the same
    distribution as the symmetric square root.
    """
    Hw = iid_channel(rng, n_sc, B, U)
    LB = np.linalg.cholesky(exp_corr(B, rho_bs))
    LU = np.linalg.cholesky(exp_corr(U, rho_ue))
    return LB[None] @ Hw @ LU.T[None]


# --------------------------------------------------------------------------
# symbols (the generator's own Gray square-QAM mapper)
# --------------------------------------------------------------------------

def _pam_levels_gray(bits_per_axis: int) -> tuple[np.ndarray, np.ndarray]:
    """Levels 2j-(L-1), j=0..L-1, and the integer Gray label of each level."""
    L = 1 << bits_per_axis
    j = np.arange(L)
    return (2 * j - (L - 1)).astype(np.float64), j ^ (j >> 1)


def qam_map(bits: np.ndarray, m: int, es: float = 1.0) -> np.ndarray:
    """Map bits (..., m) to square M-QAM symbols with average energy ``es``.

    Bits [0, m/2) select the in-phase level (MSB first) and bits [m/2, m) the
    quadrature level; the per-axis label is the Gray code of the level index,
    so bit value 0 of QPSK maps to the negative level.
    """
    if m % 2 or m < 2:
        raise ValueError("square QAM needs an even number of bits per symbol")
    h = m // 2
    levels, labels = _pam_levels_gray(h)
    inv = np.empty_like(labels)
    inv[labels] = np.arange(labels.size)          # Gray label -> level index
    w = 1 << np.arange(h - 1, -1, -1)
    li = (bits[..., :h] * w).sum(-1)
    lq = (bits[..., h:] * w).sum(-1)
    M = 1 << m
    scale = math.sqrt(es * 3.0 / (2.0 * (M - 1)))
    return scale * (levels[inv[li]] + 1j * levels[inv[lq]])


def random_bits(rng: np.random.Generator, shape: tuple, m: int) -> np.ndarray:
    return rng.integers(0, 2, size=tuple(shape) + (m,), dtype=np.int8)


def awgn(rng: np.random.Generator, shape: tuple, n0: float) -> np.ndarray:
    s = math.sqrt(n0 / 2.0)
    return rng.standard_normal(shape) * s + 1j * rng.standard_normal(shape) * s


# --------------------------------------------------------------------------
# SNR convention
# --------------------------------------------------------------------------

def n0_from_snr_db(snr_db: float, U: int, B: int, es: float = 1.0,
                   definition: str = "paper") -> float:
    """Noise variance N0 for a given SNR in dB.

    "paper": the average uplink SNR is U*E_s/N0 (Sec. II-A), so
    N0 = U*E_s/SNR.  "per_user": N0 = E_s/SNR.  "per_antenna": receive SNR per
    BS antenna with CN(0,1/B) channels, N0 = U*E_s/(B*SNR).
    """
    snr = 10.0 ** (snr_db / 10.0)
    if definition == "paper":
        return U * es / snr
    if definition == "per_user":
        return es / snr
    if definition == "per_antenna":
        return U * es / (B * snr)
    raise ValueError(definition)


# --------------------------------------------------------------------------
# frames
# --------------------------------------------------------------------------

@dataclasses.dataclass
class UplinkFrame:
    H: np.ndarray          # (n_sc, B, U) complex128
    Y: np.ndarray          # (n_sc, B, S) complex128
    X: np.ndarray          # (n_sc, U, S) transmitted symbols
    bits: np.ndarray       # (n_sc, U, S, m) int8
    n0: float
    es: float
    m: int


@dataclasses.dataclass
class DownlinkFrame:
    H: np.ndarray          # (n_sc, B, U) uplink channel; H_d = H^H
    T: np.ndarray          # (n_sc, U, S)
    bits: np.ndarray
    beta: float            # precoding regularizer (0 = zero forcing)
    m: int


def uplink_frame(rng: np.random.Generator, n_sc: int, B: int, U: int, S: int,
                 m: int, snr_db: float, es: float = 1.0, channel: str = "iid",
                 rho_bs: float = 0.0, rho_ue: float = 0.0,
                 snr_definition: str = "paper") -> UplinkFrame:
    """Draw H, then bits, then noise (fixed order), and form Y = H X + N."""
    if channel == "iid":
        H = iid_channel(rng, n_sc, B, U)
    elif channel == "kronecker":
        H = kronecker_channel(rng, n_sc, B, U, rho_bs, rho_ue)
    else:
        raise ValueError(channel)
    bits = random_bits(rng, (n_sc, U, S), m)
    X = qam_map(bits, m, es)
    n0 = n0_from_snr_db(snr_db, U, B, es, snr_definition)
    N = awgn(rng, (n_sc, B, S), n0)
    Y = H @ X + N
    return UplinkFrame(H=H, Y=Y, X=X, bits=bits, n0=n0, es=es, m=m)


def downlink_frame(rng: np.random.Generator, n_sc: int, B: int, U: int, S: int,
                   m: int, snr_db: float | None, es: float = 1.0,
                   channel: str = "iid", rho_bs: float = 0.0,
                   rho_ue: float = 0.0, H: np.ndarray | None = None,
                   snr_definition: str = "paper") -> DownlinkFrame:
    """Downlink symbols; beta = N0/E_s from the same SNR rule, 0 if snr_db is None."""
    if H is None:
        if channel == "iid":
            H = iid_channel(rng, n_sc, B, U)
        else:
            H = kronecker_channel(rng, n_sc, B, U, rho_bs, rho_ue)
    bits = random_bits(rng, (n_sc, U, S), m)
    T = qam_map(bits, m, es)
    beta = 0.0 if snr_db is None else n0_from_snr_db(snr_db, U, B, es, snr_definition) / es
    return DownlinkFrame(H=H, T=T, bits=bits, beta=beta, m=m)


# --------------------------------------------------------------------------
# the workloads (sizes, value distributions) used by tests and the benchmark
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    B: int
    U: int
    n_sc: int
    S: int
    m: int
    K: int
    snr_db: tuple
    channel: str = "iid"
    rho_bs: float = 0.0
    rho_ue: float = 0.0
    scalar_f64: bool = False


WORKLOADS = {
    # 32x8, 64 subcarriers, one OFDM symbol, 16-QAM, 10 dB, K=3
    "small_32x8": Workload("small_32x8", 32, 8, 64, 1, 4, 3, (10.0,)),
    # 128x8, 1200 subcarriers x 14 symbols, 64-QAM, 0..20 dB, K=3
    "plain_128x8": Workload("plain_128x8", 128, 8, 1200, 14, 6, 3,
                            tuple(float(s) for s in range(0, 21, 2))),
    # 128x16 and 128x32, 1200 x 14, 64-QAM, 15 dB, K=4
    "mixed_128x16": Workload("mixed_128x16", 128, 16, 1200, 14, 6, 4, (15.0,)),
    "mixed_128x32": Workload("mixed_128x32", 128, 32, 1200, 14, 6, 4, (15.0,)),
    # 256x32 Kronecker-correlated, 3300 x 14, 256-QAM, 25 dB, K=6, FP64 scalars
    "corr_256x32": Workload("corr_256x32", 256, 32, 3300, 14, 8, 6, (25.0,),
                            channel="kronecker", rho_bs=0.5, rho_ue=0.2,
                            scalar_f64=True),
}


# --------------------------------------------------------------------------
# serving stream: Poisson arrivals of mixed-shape uplink/downlink frames
# --------------------------------------------------------------------------

@dataclasses.dataclass
class StreamChannel:
    ch_id: int
    B: int
    U: int
    n_sc: int
    H: np.ndarray           # (n_sc, B, U)


@dataclasses.dataclass
class StreamFrame:
    t_arrival: float        # seconds from stream start
    ch_id: int
    uplink: bool
    m: int                  # bits per symbol
    snr_db: float


def serving_stream(rng: np.random.Generator, n_channels: int, n_frames: int, rate: float,
                   B_set=(64, 128, 256), U_set=(8, 16, 32), n_sc_range=(300, 1200),
                   m_set=(4, 6, 8), snr_range=(5.0, 25.0), uplink_share: float = 0.5):
    """Channels with B, U drawn from the sets and n_sc uniform in the range;
    frames with exponential inter-arrival times at `rate` frames/s (rate <= 0:
    all arrive at t = 0), a channel uniformly at random, QAM and SNR drawn
    per frame, uplink with probability `uplink_share`."""
    chans = []
    for c in range(n_channels):
        B = int(rng.choice(B_set))
        U = int(rng.choice(U_set))
        n_sc = int(rng.integers(n_sc_range[0], n_sc_range[1] + 1))
        chans.append(StreamChannel(c, B, U, n_sc, iid_channel(rng, n_sc, B, U)))
    return chans, serving_frames(rng, n_channels, n_frames, rate, m_set, snr_range,
                                 uplink_share)


def serving_frames(rng: np.random.Generator, n_channels: int, n_frames: int, rate: float,
                   m_set=(4, 6, 8), snr_range=(5.0, 25.0), uplink_share: float = 0.5):
    """The frames of a serving stream over existing channels 0 .. n_channels-1
    (see serving_stream)."""
    gaps = (rng.exponential(1.0 / rate, n_frames) if rate > 0 else np.zeros(n_frames))
    t = np.cumsum(gaps) - (gaps[0] if n_frames else 0.0)
    return [StreamFrame(float(t[i]), int(rng.integers(n_channels)),
                        bool(rng.random() < uplink_share), int(rng.choice(m_set)),
                        float(rng.uniform(*snr_range))) for i in range(n_frames)]

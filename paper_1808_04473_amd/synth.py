"""Seeded synthetic uplink workloads (inputs only).

This module draws the inputs of the massive MU-MIMO uplink y = H s0 + n
(Section II-A, eq. (iorelation)): i.i.d. Rayleigh-fading channel matrices
(Definition 2: entries CN(0, 1/B)), transmit symbols uniform over a
zero-mean square QAM constellation normalised to E_s = 1 (eq. (prior)),
and circularly-symmetric Gaussian noise of variance N0 per complex entry.
N0 follows the paper's receive-SNR definition SNR = beta*E_s/N0 with
beta = U/B (Section V-A).

It is the only code shared by the FP64 oracle tests and the GPU path, and it
holds none of the equaliser's arithmetic: no Gram matrix, matched filter,
solve or fusion is computed here.  Every array it returns is what both sides
consume: H and y are complex64, N0 is a float32-representable value.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 180804473 * 10

# Per-axis amplitude levels of the square constellations, before normalisation.
_LEVELS = {
    "qpsk": np.array([-1.0, 1.0]),
    "16qam": np.array([-3.0, -1.0, 1.0, 3.0]),
    "64qam": np.array([-7.0, -5.0, -3.0, -1.0, 1.0, 3.0, 5.0, 7.0]),
}


def constellation(name: str) -> np.ndarray:
    """All points of a square QAM constellation with E|s|^2 = 1 (complex128)."""
    lv = _LEVELS[name]
    pts = (lv[:, None] + 1j * lv[None, :]).reshape(-1)
    return pts / math.sqrt(np.mean(np.abs(pts) ** 2))


def noise_variance(U: int, B: int, snr_db: float, es: float = 1.0) -> float:
    """N0 from SNR = beta*E_s/N0, beta = U/B, rounded to float32."""
    beta = U / B
    return float(np.float32(beta * es / 10.0 ** (snr_db / 10.0)))


def uniform_partition(B: int, C: int) -> np.ndarray:
    """Contiguous equal-size cluster offsets off[0..C] (B divisible by C)."""
    if B % C:
        raise ValueError("B must be divisible by C for a uniform partition")
    return np.arange(C + 1, dtype=np.int32) * (B // C)


@dataclass
class Batch:
    """One batch of W independent systems sharing (B, U, partition, N0)."""

    H: np.ndarray            # [W][B][U] complex64
    y: np.ndarray            # [W][B] complex64
    s: np.ndarray            # [W][U] complex64 transmitted symbols
    n0: float                # float32-representable noise variance
    cluster_off: np.ndarray  # [C+1] int32
    es: float = 1.0

    @property
    def W(self) -> int:
        return self.H.shape[0]

    @property
    def B(self) -> int:
        return self.H.shape[1]

    @property
    def U(self) -> int:
        return self.H.shape[2]

    @property
    def C(self) -> int:
        return len(self.cluster_off) - 1


def _rayleigh(rng: np.random.Generator, shape, B: int) -> np.ndarray:
    sd = np.float32(math.sqrt(1.0 / (2.0 * B)))
    re = rng.standard_normal(shape, dtype=np.float32) * sd
    im = rng.standard_normal(shape, dtype=np.float32) * sd
    out = np.empty(shape, dtype=np.complex64)
    out.real = re
    out.imag = im
    return out


def make_batch(W: int, B: int, U: int, C: int, snr_db: float, mod: str,
               seed: int, cluster_off=None) -> Batch:
    """Draw W systems: H ~ CN(0,1/B) i.i.d., s uniform over `mod`, y = H s + n.

    y is formed in double precision from the complex64 H and then rounded to
    complex64, so both consumers see exactly the same operands.
    """
    rng = np.random.default_rng(seed)
    H = _rayleigh(rng, (W, B, U), B)
    pts = constellation(mod)
    s = pts[rng.integers(0, len(pts), size=(W, U))]
    n0 = noise_variance(U, B, snr_db)
    sdn = math.sqrt(n0 / 2.0)
    noise = (rng.standard_normal((W, B)) + 1j * rng.standard_normal((W, B))) * sdn
    y = np.matmul(H.astype(np.complex128), s[:, :, None])[:, :, 0] + noise
    off = uniform_partition(B, C) if cluster_off is None else np.asarray(cluster_off, np.int32)
    return Batch(H=H, y=y.astype(np.complex64), s=s.astype(np.complex64), n0=n0,
                 cluster_off=off)


# The five workloads: shapes, modulation and SNR.  `seed_id` selects the seed.
CONFIGS = {
    1: dict(B=32, C=2, U=4, W=64, mod="qpsk", snrs=(10.0,)),
    2: dict(B=256, C=8, U=16, W=1200, mod="16qam", snrs=(0.0, 10.0, 20.0)),
    3: dict(B=1024, C=16, U=32, W=1200, mod="16qam", snrs=(0.0, 10.0, 20.0)),
    5: dict(B=256, C=8, U=16, W=1200, mod="16qam", snrs=(10.0,)),
}


def config_batch(cfg: int, snr_db: float | None = None, frame: int = 0,
                 W: int | None = None) -> Batch:
    """Batch of workload `cfg` (1, 2, 3 or 5); frame f uses seed + 1000 f."""
    c = CONFIGS[cfg]
    snr = c["snrs"][0] if snr_db is None else snr_db
    seed = BASE_SEED + cfg + 1000 * frame + int(round(snr * 7))
    return make_batch(W or c["W"], c["B"], c["U"], c["C"], snr, c["mod"], seed)


@dataclass
class SymbolBatch:
    """W channel matrices, each shared by S receive vectors (OFDM symbols of
    one coherence interval): Y[w, s] = H[w] x[w, s] + n[w, s]."""

    H: np.ndarray            # [W][B][U] complex64
    Y: np.ndarray            # [W][S][B] complex64
    x: np.ndarray            # [W][S][U] complex64 transmitted symbols
    n0: float
    cluster_off: np.ndarray  # [C+1] int32
    es: float = 1.0


def make_symbol_batch(W: int, B: int, U: int, C: int, S: int, snr_db: float, mod: str,
                      seed: int, cluster_off=None) -> SymbolBatch:
    """As make_batch, with S independent symbol vectors and noise draws per
    channel matrix (formed in double precision, rounded to complex64)."""
    rng = np.random.default_rng(seed)
    H = _rayleigh(rng, (W, B, U), B)
    pts = constellation(mod)
    x = pts[rng.integers(0, len(pts), size=(W, S, U))]
    n0 = noise_variance(U, B, snr_db)
    sdn = math.sqrt(n0 / 2.0)
    noise = (rng.standard_normal((W, S, B)) + 1j * rng.standard_normal((W, S, B))) * sdn
    Y = np.matmul(x.astype(np.complex128), np.swapaxes(H.astype(np.complex128), 1, 2)) + noise
    off = uniform_partition(B, C) if cluster_off is None else np.asarray(cluster_off, np.int32)
    return SymbolBatch(H=H, Y=Y.astype(np.complex64), x=x.astype(np.complex64), n0=n0,
                       cluster_off=off)


def symbols_for_channels(H: np.ndarray, S: int, snr_db: float, mod: str, seed: int):
    """S receive vectors per given channel matrix: (Y [W][S][B], x [W][S][U]),
    Y = H x + n in complex64 arithmetic (for large throughput workloads)."""
    W, B, U = H.shape
    rng = np.random.default_rng(seed)
    pts = constellation(mod).astype(np.complex64)
    x = pts[rng.integers(0, len(pts), size=(W, S, U))]
    sdn = np.float32(math.sqrt(noise_variance(U, B, snr_db) / 2.0))
    Y = np.matmul(x, np.swapaxes(H, 1, 2))
    Y.real += rng.standard_normal((W, S, B), dtype=np.float32) * sdn
    Y.imag += rng.standard_normal((W, S, B), dtype=np.float32) * sdn
    return np.ascontiguousarray(Y, dtype=np.complex64), x


def config_symbol_batch(cfg: int, nsym: int = 14, snr_db: float | None = None, frame: int = 0,
                        W: int | None = None) -> SymbolBatch:
    """Workload `cfg` with nsym OFDM symbols per channel matrix."""
    c = CONFIGS[cfg]
    snr = c["snrs"][0] if snr_db is None else snr_db
    seed = BASE_SEED + 50 + cfg + 1000 * frame + int(round(snr * 7))
    return make_symbol_batch(W or c["W"], c["B"], c["U"], c["C"], nsym, snr, c["mod"], seed)


# ---------------------------------------------------------------------------
# Ragged workload: thousands of independent systems of uneven shape.
# ---------------------------------------------------------------------------
RAGGED_BC = (16, 24, 32, 48, 64)
RAGGED_U = (8, 16, 24, 32)


@dataclass
class RaggedBatch:
    """Independent systems packed back to back in flat pools.

    System k owns H_pool[h_off[k] : h_off[k] + B_k*U_k] (row-major [B_k][U_k]),
    y_pool[y_off[k] : y_off[k] + B_k] and z_pool[z_off[k] : z_off[k] + U_k];
    its clusters are cluster_sizes[clus_first[k] : clus_first[k] + C_k].
    """

    H_pool: np.ndarray
    y_pool: np.ndarray
    s_pool: np.ndarray
    B: np.ndarray
    U: np.ndarray
    C: np.ndarray
    n0: np.ndarray
    h_off: np.ndarray
    y_off: np.ndarray
    z_off: np.ndarray
    clus_first: np.ndarray
    cluster_sizes: np.ndarray
    es: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def nsys(self) -> int:
        return len(self.B)

    def system(self, k: int):
        """(H [B][U] c64, y [B] c64, n0, cluster offsets [C+1]) of system k."""
        B, U, C = int(self.B[k]), int(self.U[k]), int(self.C[k])
        H = self.H_pool[self.h_off[k]:self.h_off[k] + B * U].reshape(B, U)
        y = self.y_pool[self.y_off[k]:self.y_off[k] + B]
        sizes = self.cluster_sizes[self.clus_first[k]:self.clus_first[k] + C]
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
        return H, y, float(self.n0[k]), off


def make_ragged(nsys: int = 4096, snr_db: float = 15.0, mod: str = "64qam",
                seed: int = BASE_SEED + 4) -> RaggedBatch:
    """U uniform over {8,16,24,32}; then C uniform in 2..16; then each B_c
    uniform over {16,24,32,48,64} restricted to B_c >= U."""
    rng = np.random.default_rng(seed)
    pts = constellation(mod)
    Us = rng.choice(RAGGED_U, size=nsys)
    Cs = rng.integers(2, 17, size=nsys)
    sizes, Bs = [], []
    for k in range(nsys):
        allowed = [b for b in RAGGED_BC if b >= Us[k]]
        bc = rng.choice(allowed, size=Cs[k])
        sizes.append(bc)
        Bs.append(int(bc.sum()))
    Bs = np.array(Bs, np.int64)
    Us = Us.astype(np.int64)
    h_off = np.concatenate([[0], np.cumsum(Bs * Us)[:-1]]).astype(np.int64)
    y_off = np.concatenate([[0], np.cumsum(Bs)[:-1]]).astype(np.int64)
    z_off = np.concatenate([[0], np.cumsum(Us)[:-1]]).astype(np.int64)
    clus_first = np.concatenate([[0], np.cumsum(Cs)[:-1]]).astype(np.int64)
    H_pool = np.empty(int((Bs * Us).sum()), np.complex64)
    y_pool = np.empty(int(Bs.sum()), np.complex64)
    s_pool = np.empty(int(Us.sum()), np.complex64)
    n0 = np.empty(nsys, np.float32)
    for k in range(nsys):
        B, U = int(Bs[k]), int(Us[k])
        H = _rayleigh(rng, (B, U), B)
        s = pts[rng.integers(0, len(pts), size=U)]
        n0k = noise_variance(U, B, snr_db)
        sdn = math.sqrt(n0k / 2.0)
        nz = (rng.standard_normal(B) + 1j * rng.standard_normal(B)) * sdn
        y = H.astype(np.complex128) @ s + nz
        H_pool[h_off[k]:h_off[k] + B * U] = H.reshape(-1)
        y_pool[y_off[k]:y_off[k] + B] = y.astype(np.complex64)
        s_pool[z_off[k]:z_off[k] + U] = s.astype(np.complex64)
        n0[k] = n0k
    return RaggedBatch(H_pool=H_pool, y_pool=y_pool, s_pool=s_pool, B=Bs.astype(np.int32),
                       U=Us.astype(np.int32), C=Cs.astype(np.int32), n0=n0,
                       h_off=h_off, y_off=y_off, z_off=z_off,
                       clus_first=clus_first,
                       cluster_sizes=np.concatenate(sizes).astype(np.int32))

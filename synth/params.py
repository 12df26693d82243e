"""Radio configuration and seeded draws of scene parameters.

Distributions follow the workload recipes: relative permittivity uniform in
[2, 10], conductivity log-uniform in [1e-3, 1] S/m, scattering coefficient 0
for plain forward runs and uniform in [0, 0.5] for calibration targets,
element gains with magnitude in [0.8, 1.2] and phase in [-pi/4, pi/4].
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Radio:
    """OFDM grid and antenna configuration.

    Subcarrier n (storage index 0..n_sc-1) sits at f_n = fc + (n - n_sc//2)*df
    with df = bandwidth / n_sc (Sec. II-A, discrete CFR: n runs from -N/2 to
    N/2-1 around the carrier, W = N*df; for odd N the carrier is the middle
    subcarrier).  The Tx is a uniform linear array of
    n_elem isotropic elements with half-wavelength spacing along `ula_axis`,
    centred on the Tx position; the Rx is one isotropic element.  zeta_* are
    polarisation slant angles (Sec. II-B, polarisation model), 0 = vertical.
    """
    fc: float = 3.5e9
    bandwidth: float = 50e6
    n_sc: int = 256
    n_elem: int = 1
    ula_axis: tuple = (1.0, 0.0, 0.0)
    zeta_tx: float = 0.0
    zeta_rx: float = 0.0

    @property
    def df(self) -> float:
        return self.bandwidth / self.n_sc

    def freqs(self) -> np.ndarray:
        n = np.arange(self.n_sc, dtype=np.float64)
        return self.fc + (n - self.n_sc // 2) * self.df


def draw_materials(rng: np.random.Generator, n_mat: int, with_scattering: bool):
    """Seeded material draw: eps_r ~ U[2,10], sigma ~ logU[1e-3,1] S/m,
    S ~ U[0,0.5] when `with_scattering`, else S = 0."""
    eps_r = rng.uniform(2.0, 10.0, n_mat)
    sigma = 10.0 ** rng.uniform(-3.0, 0.0, n_mat)
    if with_scattering:
        s = rng.uniform(0.0, 0.5, n_mat)
    else:
        s = np.zeros(n_mat)
    return eps_r, sigma, s


# Raw value that stands for S = 0 in the logistic parametrisation: its
# sigmoid is 4e-18, so sqrt(1 - S^2) rounds to exactly 1 in FP32 and FP64.
RAW_S_ZERO = -40.0


def materials_to_raw(eps_r, sigma, s) -> np.ndarray:
    """Raw per-material parameters u with eps_r = 1 + e^u0, sigma = e^u1,
    S = logistic(u2) (the trainable-material parametrisation of Sec. III-C
    with one-dimensional embeddings and unit read-out).  Returned as
    float32 [n_mat, 3], the layout the libraries take."""
    eps_r = np.asarray(eps_r, np.float64)
    sigma = np.asarray(sigma, np.float64)
    s = np.asarray(s, np.float64)
    u0 = np.log(eps_r - 1.0)
    u1 = np.log(sigma)
    with np.errstate(divide="ignore"):
        u2 = np.where(s > 0, np.log(s) - np.log1p(-s), RAW_S_ZERO)
    return np.stack([u0, u1, u2], axis=1).astype(np.float32)


def draw_gains(rng: np.random.Generator, n_elem: int) -> np.ndarray:
    """Hidden element gains g_m = A_m e^{j phi_m}, A ~ U[0.8,1.2],
    phi ~ U[-pi/4, pi/4]; complex64 [n_elem]."""
    amp = rng.uniform(0.8, 1.2, n_elem)
    ph = rng.uniform(-np.pi / 4, np.pi / 4, n_elem)
    return (amp * np.exp(1j * ph)).astype(np.complex64)


@dataclass
class Workload:
    """A named workload: scene recipe, radio grid and sizes."""
    name: str
    radio: Radio
    n_rx: int
    max_depth: int
    n_mat: int
    seed: int
    extra: dict = field(default_factory=dict)


MLP_SHAPES = [(128, 51), (128, 128), (128, 128), (128, 128), (3, 128)]


def mlp_init(rng: np.random.Generator, out_bias=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Seeded MLP parameters, packed W0, b0, ..., W4, b4 (row-major out x in):
    uniform in +-1/sqrt(fan_in) for weights and hidden biases; the three
    output biases are set to `out_bias`.  float32 [56579]."""
    parts = []
    for li, (o, i) in enumerate(MLP_SHAPES):
        bound = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-bound, bound, o * i))
        if li == len(MLP_SHAPES) - 1:
            parts.append(np.asarray(out_bias, np.float64))
        else:
            parts.append(rng.uniform(-bound, bound, o))
    return np.concatenate(parts).astype(np.float32)


def draw_path_coefficients(rng: np.random.Generator, tau: np.ndarray, fc: float):
    """Seeded stand-ins for per-path coefficients, for tests of the stages
    after the field computation at sizes where computing the fields is not
    the point: a_i with magnitude lambda/(4 pi c tau_i) times U[0.05, 1] and
    a uniform phase, psi_i uniform in [-pi, pi].  Returns (a complex64 [P],
    psi float32 [P])."""
    c0 = 299792458.0
    tau = np.asarray(tau, np.float64)
    amp = (c0 / fc) / (4.0 * np.pi * c0 * tau) * rng.uniform(0.05, 1.0, tau.shape)
    a = amp * np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, tau.shape))
    psi = rng.uniform(-np.pi, np.pi, tau.shape)
    return a.astype(np.complex64), psi.astype(np.float32)


def draw_target_cfr(rng: np.random.Generator, link_power: np.ndarray, n_elem: int, n_sc: int):
    """Seeded stand-in target CFRs c64 [L, n_elem, n_sc]: circular Gaussian
    entries whose variance per link is link_power[l]."""
    L = len(link_power)
    s = np.sqrt(np.asarray(link_power, np.float64) / 2.0)[:, None, None]
    re = rng.standard_normal((L, n_elem, n_sc), dtype=np.float32)
    im = rng.standard_normal((L, n_elem, n_sc), dtype=np.float32)
    return ((re + 1j * im) * s).astype(np.complex64)

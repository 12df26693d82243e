"""The paper's own calibration loss, scale estimate and evaluation metrics
(oracle, FP64).  Test infrastructure only: imported by tests, the smoke
check and the CPU baseline of the benchmark, never by the library path.

  * CIR taps h[l], l = -N/2 .. N/2-1, by the centred 1/sqrt(N) IDFT of the
    OFDM CFR (Sec. II-A, the same definition as channel.cir); p_l = |h[l]|^2
  * total gain P = sum_l p_l (Eq. channel_gain)
  * RMS delay spread (Eq. delay_spread): with the mean tap
    tau_bar = sum_l l p_l / P (in taps), tau_RMS = sqrt(sum_l ((l - tau_bar)
    / W)^2 p_l / P) seconds, W = N * df the bandwidth
  * SMAPE l(x, y) = |x - y| / (x + y) (Eq. smape)
  * per-example loss l(tau_RMS, tau_RMS^) + l(P, P^) (Eq. loss); the batch
    loss of Algorithm 1 is its mean over the examples
  * least-squares scale alpha^ = sum_b P_b P^_b / sum_b P_b^2 (Eq. alpha_hat)
    and its exponential moving average alpha_i = delta alpha_{i-1} + (1 -
    delta) alpha^_i with alpha_0 = alpha^_1 (Eq. scaling_param); the
    measured CIRs are scaled by sqrt(alpha_i), i.e. their gains by alpha_i
  * evaluation metrics of Sec. IV-C: per measurement point, gains and delay
    spreads averaged over its receive antennas, ALE = |Pbar_dB - Pbar^_dB|,
    RAE = |taubar - taubar^| / taubar.

Readings where the paper leaves a choice (each listed with the design notes):
  * an example is one CIR, i.e. one (link, array element) row of N
    subcarriers; the batch mean runs over all rows;
  * a row with P = 0 has tau_RMS = 0; l(0, 0) = 0;
  * alpha enters the loss as a constant (it is estimated, not learned) and
    alpha^ uses the predictions of the current batch;
  * derivatives at the kinks of |.| and sqrt are torch's (sign(0) = 0,
    and the delay-spread term is cut when its variance is 0).
"""
import torch

from .channel import cir
from .em import f64


def tap_index(N):
    """Delay index l = -N/2 .. N/2-1 in the storage order of channel.cir."""
    return torch.arange(N, dtype=f64) - N // 2


def pdp_centred(H):
    """p_l = |h[l]|^2 over the last axis, l = -N/2 .. N/2-1 at position l + N/2."""
    return torch.abs(cir(H)) ** 2


def gain_and_delay_spread(H, bandwidth):
    """(P, tau_RMS) of every CIR row of H [..., N]; tau_RMS in seconds."""
    N = H.shape[-1]
    p = pdp_centred(H)
    ell = tap_index(N)
    P = p.sum(-1)
    safe = torch.where(P > 0, P, torch.ones_like(P))
    w = p / safe[..., None]                     # p_l / P
    tau_bar = (ell * w).sum(-1)                 # mean tap
    var = ((((ell - tau_bar[..., None]) / bandwidth) ** 2) * w).sum(-1)
    pos = var > 0
    tau = torch.where(pos, torch.sqrt(torch.where(pos, var, torch.ones_like(var))),
                      torch.zeros_like(var))
    tau = torch.where(P > 0, tau, torch.zeros_like(tau))
    return P, tau


def smape(x, y):
    """|x - y| / (x + y), 0 where x + y = 0 (Eq. smape)."""
    s = x + y
    pos = s > 0
    return torch.where(pos, torch.abs(x - y) / torch.where(pos, s, torch.ones_like(s)),
                       torch.zeros_like(s))


def example_losses(P_tgt, tau_tgt, P_hat, tau_hat, alpha=1.0, w_tau=1.0, w_gain=1.0):
    """Per-example terms (Eq. loss) against measurements scaled by alpha:
    returns (w_tau l(tau, tau^) + w_gain l(alpha P, P^), l_tau, l_gain)."""
    l_tau = smape(tau_tgt, tau_hat)
    l_gain = smape(alpha * P_tgt, P_hat)
    return w_tau * l_tau + w_gain * l_gain, l_tau, l_gain


def batch_loss(H_pred, P_tgt, tau_tgt, bandwidth, alpha=1.0, w_tau=1.0, w_gain=1.0):
    """Mean over all CIR rows of the per-example loss; returns (L, mean
    l_tau, mean l_gain).  alpha is a plain number (no gradient)."""
    P_hat, tau_hat = gain_and_delay_spread(H_pred, bandwidth)
    tot, lt, lg = example_losses(P_tgt, tau_tgt, P_hat, tau_hat, alpha, w_tau, w_gain)
    return tot.mean(), lt.mean(), lg.mean()


def alpha_hat(P_meas, P_pred):
    """Least-squares scale between measured and predicted gains (Eq. alpha_hat)."""
    P_meas = torch.as_tensor(P_meas, dtype=f64)
    P_pred = torch.as_tensor(P_pred, dtype=f64)
    return float((P_meas * P_pred).sum() / (P_meas * P_meas).sum())


def alpha_ema(alpha_prev, a_hat, delta, first):
    """One step of Eq. scaling_param; on the first step alpha_0 = alpha^_1."""
    prev = a_hat if first else alpha_prev
    return delta * prev + (1.0 - delta) * a_hat


def to_db(x):
    return 10.0 * torch.log10(x)


def ale_rae(P_meas, tau_meas, P_pred, tau_pred, n_elem, scale=1.0):
    """Per measurement point (a link with n_elem CIR rows): ALE in dB and
    RAE of the antenna-averaged gain and delay spread (Sec. IV-C).  The
    measured gains are multiplied by `scale` (the estimated alpha)."""
    Pm = (scale * P_meas.reshape(-1, n_elem)).mean(-1)
    Pp = P_pred.reshape(-1, n_elem).mean(-1)
    tm = tau_meas.reshape(-1, n_elem).mean(-1)
    tp = tau_pred.reshape(-1, n_elem).mean(-1)
    return torch.abs(to_db(Pm) - to_db(Pp)), torch.abs(tm - tp) / tm

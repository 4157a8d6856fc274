"""Closed forms used to pin the oracle (no oracle code is used here).

* One-link SU(3) integral.  With weight exp((b/3) Re Tr U) and Haar measure,
  u(b) = d/db ln z(b) = <1/3 Re Tr U>, where by Weyl's integration formula
  z(b) = int dth1 dth2 |Delta(e^{i th})|^2 exp((b/3) sum_k cos th_k),
  th3 = -th1 - th2, |Delta|^2 = prod_{i<j} 4 sin^2((th_i - th_j)/2).
  The integrand is smooth and periodic, so the uniform-grid rule converges
  spectrally.  u(b) is also the leading strong-coupling value of the mean
  plaquette of the Wilson action (corrections start at O(u^5)), and the
  expectation of 1/3 Re Tr(U A)/c for one link in a fixed staple A = c G,
  G in SU(3).

* Kennedy-Pendleton SU(2) sampler.  The target density of a0 on [-1, 1] is
  sqrt(1 - a0^2) exp(alpha a0), with normaliser pi I1(alpha)/alpha and mean
  I2(alpha)/I1(alpha).  One attempt proposes lambda^2 ~ Gamma(3/2)/(2 alpha)
  and accepts with probability sqrt(1 - lambda^2); its acceptance probability
  is sqrt(2 pi alpha) exp(-alpha) I1(alpha).
"""
import numpy as np
from scipy import integrate, special


def weyl_u(b, n=256):
    th = 2 * np.pi * np.arange(n) / n
    t1, t2 = np.meshgrid(th, th, indexing="ij")
    t3 = -t1 - t2
    vdm = (16 * np.sin((t1 - t2) / 2) ** 2 * 4 * np.sin((t1 - t3) / 2) ** 2
           * np.sin((t2 - t3) / 2) ** 2)
    s = (np.cos(t1) + np.cos(t2) + np.cos(t3)) / 3.0
    w = vdm * np.exp(b * s)
    return float((w * s).sum() / w.sum())


def kp_density(a0, alpha):
    return np.sqrt(1 - a0 ** 2) * np.exp(alpha * a0) * alpha / (np.pi * special.i1(alpha))


def kp_normaliser(alpha):
    return np.pi * special.i1(alpha) / alpha


def kp_mean(alpha):
    return special.iv(2, alpha) / special.iv(1, alpha)


def kp_bin_probs(edges, alpha):
    # integrate the unnormalised density scaled by exp(-alpha) for stability
    f = lambda x: np.sqrt(max(0.0, 1 - x * x)) * np.exp(alpha * (x - 1))
    probs = np.array([integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-12)[0]
                      for lo, hi in zip(edges[:-1], edges[1:])])
    total = np.pi * special.ive(1, alpha) / alpha
    return probs / total, probs.sum() / total


def kp_acceptance(alpha):
    return float(np.sqrt(2 * np.pi * alpha) * special.ive(1, alpha))


def batch_mean_error(x, nbins=20):
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // nbins
    b = x[: m * nbins].reshape(nbins, m).mean(axis=1)
    return float(x.mean()), float(b.std(ddof=1) / np.sqrt(nbins))

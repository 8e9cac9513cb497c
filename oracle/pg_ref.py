"""Reference Polya-Gamma draws for the omega update of the Gibbs sampler.

Test infrastructure only: see the package docstring.

The Gibbs cycle of Supplement S1 (step 3) draws omega_i ~ PG(1, x_i^T beta)
and the Gaussian pseudo-response is z_i = (y_i - 1/2) / omega_i (eq.
pg_augmented_likelihood).  The paper cites Polson, Scott & Windle (2013) for
the Polya-Gamma law and gives no sampler; this module restates the exact
sampler of Devroye (2009) as described by Polson, Scott & Windle, Section 4:

* PG(1, c) = J*(1, z) / 4 with z = |c| / 2.
* The density of J*(1, z) is cosh(z) exp(-z^2 x / 2) sum_n (-1)^n a_n(x), an
  alternating series whose terms decrease from n = 1 on, with two forms of
  a_n split at t = 0.64:
      x <= t:  a_n(x) = pi (n + 1/2) (2 / (pi x))^(3/2) exp(-2 (n + 1/2)^2 / x)
      x >  t:  a_n(x) = pi (n + 1/2) exp(-(n + 1/2)^2 pi^2 x / 2).
* Proposal: exp(-z^2 x / 2) a_0(x), a mixture of an exponential with rate
  K = pi^2 / 8 + z^2 / 2 on (t, inf) (mass p = pi / (2 K) exp(-K t)) and an
  inverse Gaussian IG(1/z, 1) truncated to (0, t] (mass q = 2 exp(-z)
  P_IG(X <= t)); the exponential part is taken with probability p / (p + q),
  evaluated from log p and log q (both masses underflow at large z).
* Acceptance: with V uniform, Y = V a_0(X) is compared against the partial
  sums of the series (lower bounds after odd terms, upper after even ones).
  Both sides are divided by a_0(X) > 0, which leaves every decision the
  same and keeps the test defined where a_0 itself underflows (tilts |c|
  beyond ~2000): V against 1 - a_1/a_0 + a_2/a_0 - ..., with
      x <= t:  a_n/a_0 = (2n + 1) exp(-2 n (n + 1) / x)
      x >  t:  a_n/a_0 = (2n + 1) exp(-n (n + 1) pi^2 x / 2).

Random numbers: element i's k-th uniform is word k mod 4 of the Philox4x64-10
block with counter (i, 2 | (k div 4) << 8, chain, draw) and key (seed, 0),
mapped to ((w >> 11) + 1/2) 2^-53 in (0, 1).  Stream word 2 (low byte) is the
Polya-Gamma stream beside eta (0) and delta (1).  Within one proposal the
uniforms are taken in this order: the mixture choice; then either the
exponential (right piece) or the truncated inverse Gaussian's (below); then
V.  The truncated inverse Gaussian with mean mu = 1/z:
* mu > t (z < 1/t, z = 0 included): the truncated Levy law by E1, E2
  exponentials until E1^2 <= 2 E2 / t, X = t / (1 + t E1)^2, then one uniform
  accepting with probability exp(-z^2 X / 2);
* mu <= t: the Michael-Schucany-Haas transform (two uniforms for a squared
  normal by Box-Muller, one to pick the root), repeated until X <= t.
Every loop is capped at 64 rounds (reached with probability far below
1e-100); a capped proposal loop returns its last candidate.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc, erfcx

from . import philox_ref as H

STREAM_PG = 2
T_SPLIT = 0.64
CAP = 64
TWO_PI = 6.283185307179586  # 2 pi rounded to double


class Uniforms:
    """Element i's uniforms u_0, u_1, ... in (0, 1)."""

    def __init__(self, seed, chain, draw, i):
        self.key = (int(seed), 0)
        self.ctr = [int(i), 0, int(chain), int(draw)]
        self.k = 0
        self.words = ()

    def __call__(self):
        w = self.k & 3
        if w == 0:
            self.ctr[1] = STREAM_PG | ((self.k >> 2) << 8)
            self.words = H.philox4x64_scalar(self.ctr, self.key)
        self.k += 1
        return ((self.words[w] >> 11) + 0.5) * 2.0 ** -53


def a_n(n, x):
    """Term n of the alternating series of the J*(1, 0) density."""
    h = n + 0.5
    if x <= T_SPLIT:
        return math.pi * h * (2.0 / (math.pi * x)) ** 1.5 * math.exp(-2.0 * h * h / x)
    return math.pi * h * math.exp(-h * h * math.pi ** 2 * x / 2.0)


def a_ratio(n, x):
    """a_n(x) / a_0(x), the series term relative to the leading one."""
    k = float(n * (n + 1))
    if x <= T_SPLIT:
        return (2 * n + 1) * math.exp(-2.0 * k / x)
    return (2 * n + 1) * math.exp(-k * math.pi ** 2 * x / 2.0)


def mixture_masses(z):
    """(p, q): masses of the exponential and truncated inverse Gaussian parts
    of the proposal.  q = 2 exp(-z) [Phi((z t - 1)/sqrt t) + exp(2 z)
    Phi(-(z t + 1)/sqrt t)], the second term written with erfcx so that it
    neither overflows nor underflows for large z."""
    t = T_SPLIT
    K = math.pi ** 2 / 8.0 + z * z / 2.0
    p = math.pi / (2.0 * K) * math.exp(-K * t)
    r = math.sqrt(2.0 * t)
    q = (math.exp(-z) * float(erfc((1.0 - z * t) / r))
         + float(erfcx((1.0 + z * t) / r)) * math.exp(-z * z * t / 2.0 - 1.0 / (2.0 * t)))
    return p, q


def right_probability(z):
    """p / (p + q), the chance of the exponential part, from the masses'
    logarithms: 1 / (1 + exp(log q - log p)), log q the log-sum of its two
    terms, so that it stays defined where p and q both underflow."""
    t = T_SPLIT
    K = math.pi ** 2 / 8.0 + z * z / 2.0
    lp = math.log(math.pi / (2.0 * K)) - K * t
    r = math.sqrt(2.0 * t)
    l1 = -z + math.log(float(erfc((1.0 - z * t) / r)))
    l2 = math.log(float(erfcx((1.0 + z * t) / r))) - z * z * t / 2.0 - 1.0 / (2.0 * t)
    hi, lo = (l1, l2) if l1 >= l2 else (l2, l1)
    lq = hi + math.log1p(math.exp(lo - hi))
    d = lq - lp
    return 0.0 if d > 700.0 else 1.0 / (1.0 + math.exp(d))


def truncated_ig(z, u):
    """A draw of IG(1/z, 1) restricted to (0, t] (z = 0: the Levy law)."""
    t = T_SPLIT
    x = t
    if z < 1.0 / t:
        for _ in range(CAP):
            for _ in range(CAP):
                e1 = -math.log(u())
                e2 = -math.log(u())
                if e1 * e1 <= 2.0 * e2 / t:
                    break
            x = t / (1.0 + t * e1) ** 2
            if u() <= math.exp(-z * z * x / 2.0):
                break
        return x
    mu = 1.0 / z
    for _ in range(CAP):
        u1, u2 = u(), u()
        cs = math.cos(TWO_PI * u2)
        y = -2.0 * math.log(u1) * cs * cs
        x = mu + 0.5 * mu * mu * y - 0.5 * mu * math.sqrt(4.0 * mu * y + (mu * y) ** 2)
        if u() > mu / (mu + x):
            x = mu * mu / x
        if x <= t:
            break
    return x


def pg1_draw(c, u):
    """One PG(1, c) draw from the uniform source u (Devroye's J*(1, |c|/2),
    divided by 4)."""
    z = 0.5 * abs(float(c))
    t = T_SPLIT
    K = math.pi ** 2 / 8.0 + z * z / 2.0
    right = right_probability(z)
    x = t
    for _ in range(CAP):
        if u() < right:
            x = t - math.log(u()) / K
        else:
            x = truncated_ig(z, u)
        s = 1.0  # partial sums over a_0(x)
        y = u()
        accepted = False
        for n in range(1, CAP):
            if n & 1:
                s -= a_ratio(n, x)
                if y < s:
                    accepted = True
                    break
            else:
                s += a_ratio(n, x)
                if y > s:
                    break
        if accepted:
            break
    return 0.25 * x


def pg_draws(seed, chain, draw, c, idx=None):
    """omega_i ~ PG(1, c_i) for the elements idx (default all), element i
    drawing from its own uniform stream."""
    c = np.asarray(c, dtype=np.float64)
    idx = np.arange(c.size) if idx is None else np.asarray(idx)
    return np.array([pg1_draw(c[i], Uniforms(seed, chain, draw, i)) for i in idx])


def pseudo_response(y, omega):
    """z_i = (y_i - 1/2) / omega_i (eq. pg_augmented_likelihood)."""
    return (np.asarray(y, dtype=np.float64) - 0.5) / np.asarray(omega, dtype=np.float64)


def pg_update(X, beta, y, seed, chain, draw, idx=None):
    """Step 3 of the Gibbs cycle and the pseudo-response it implies: psi =
    X beta, omega_i ~ PG(1, psi_i), z_i = (y_i - 1/2) / omega_i; for the
    elements idx (default all)."""
    psi = X @ np.asarray(beta, dtype=np.float64)
    omega = pg_draws(seed, chain, draw, psi, idx)
    yy = np.asarray(y)[np.arange(psi.size) if idx is None else np.asarray(idx)]
    return omega, pseudo_response(yy, omega), psi

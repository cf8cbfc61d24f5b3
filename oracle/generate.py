"""Oracle for candidate-orbit generation (Algorithm 1, GenerateOrbits).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
baseline of the benchmark; the library never imports it.

The paper draws candidate orbital parameters from given distributions
(Sec. 3).  The reading used here: a, e, i uniform in their ranges; a line of
sight uniform over a tangent-plane rectangle about a field centre; the orbit
is placed so that its geometric heliocentric position at the epoch lies on
that line of sight from the observer, with a uniform true anomaly nu and a
uniform choice between the two nodal branches.  Concretely, for one attempt:

  r    = a (1 - e^2) / (1 + e cos nu)                (conic at true anomaly nu)
  X    = O + s d,  s > 0 the far root of |O + s d| = r
  beta = asin(X_z / |X|),  lambda = atan2(X_y, X_x)   (ecliptic latitude/longitude)
  i    = max(i, |beta| (1 + 1e-9) + 1e-12)            (an orbit plane must reach beta)
  u    = asin(sin beta / sin i), replaced by pi - u when draw 6 is < 1/2
  Omega = lambda - atan2(cos i sin u, cos u),  omega = u - nu
  E    = 2 atan2(sqrt(1-e) sin(nu/2), sqrt(1+e) cos(nu/2)),  M0 = E - e sin E

An attempt whose line of sight misses the sphere is redrawn (16 attempts;
then a = NaN).

Random numbers: draw k of attempt t for orbit index j is
  U = (h >> 11) 2^-53,  h = SM(seed XOR SM(j * 1099511628211 + 16 t + k))
where SM(x) is the first output of SplitMix64 (Steele, Lea and Flood 2014)
started from state x, all arithmetic modulo 2^64.  The library implements the
same published generator on its own.
"""
from __future__ import annotations

import math

import numpy as np

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(state: int) -> int:
    """First output of SplitMix64 from the given 64-bit state."""
    z = (state + _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def uniform(seed: int, j: int, attempt: int, k: int) -> float:
    ctr = (j * 0x100000001B3 + attempt * 16 + k) & _M64
    h = splitmix64((seed & _M64) ^ splitmix64(ctr))
    return (h >> 11) * 2.0 ** -53


def sample_orbit(S: dict, j: int):
    """Elements (a, e, i, Omega, omega, M0) of orbit j of sampler S, or None."""
    c, ea, no = (np.asarray(S[k], np.float64) for k in ("center", "east", "north"))
    O = np.asarray(S["obs"], np.float64)
    for t in range(16):
        U = [uniform(S["seed"], j, t, k) for k in range(7)]
        xi = (2 * U[0] - 1) * S["half_w"]
        eta = (2 * U[1] - 1) * S["half_h"]
        d = c + xi * ea + eta * no
        d = d / math.sqrt(float(d @ d))
        a = S["a"][0] + (S["a"][1] - S["a"][0]) * U[2]
        e = S["e"][0] + (S["e"][1] - S["e"][0]) * U[3]
        inc = S["inc"][0] + (S["inc"][1] - S["inc"][0]) * U[4]
        nu = math.pi * (2 * U[5] - 1)
        r = a * (1 - e * e) / (1 + e * math.cos(nu))
        # |O + s d|^2 = r^2  ->  s^2 + 2 (O.d) s + |O|^2 - r^2 = 0
        od = float(O @ d)
        disc = od * od - float(O @ O) + r * r
        if not disc > 0:
            continue
        s = -od + math.sqrt(disc)
        if not s > 0:
            continue
        X = O + s * d
        beta = math.asin(max(-1.0, min(1.0, X[2] / math.sqrt(float(X @ X)))))
        lam = math.atan2(X[1], X[0])
        inc = max(inc, abs(beta) * (1 + 1e-9) + 1e-12)
        u = math.asin(max(-1.0, min(1.0, math.sin(beta) / math.sin(inc))))
        if U[6] < 0.5:
            u = math.pi - u
        node = lam - math.atan2(math.cos(inc) * math.sin(u), math.cos(u))
        peri = u - nu
        E = 2 * math.atan2(math.sqrt(1 - e) * math.sin(nu / 2), math.sqrt(1 + e) * math.cos(nu / 2))
        M0 = E - e * math.sin(E)
        return (a, e, inc, node % (2 * math.pi), peri % (2 * math.pi), M0)
    return None


def generate(S: dict, first: int, n: int) -> np.ndarray:
    """(n, 6) elements of orbits first .. first + n - 1 (a = NaN where all attempts missed)."""
    out = np.zeros((n, 6))
    for j in range(n):
        el = sample_orbit(S, first + j)
        if el is None:
            out[j, 0] = np.nan
        else:
            out[j] = el
    return out

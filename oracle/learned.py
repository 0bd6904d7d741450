"""Oracle: the learned hyperparameter warm start and the likelihood fit it seeds.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper fits the GP hyperparameters of each light curve by maximum
likelihood, with the trend solved linearly (Section 3.2), before the search.
The learned part trains a small 1D CNN on light curves drawn from the GP
itself to predict those hyperparameters as the starting point of that fit.
This module writes out, in FP64 and in plain loops:

* ``philox4x32_10``: the counter-based generator of Salmon, Moraes, Dror and
  Shaw (SC'11, "Parallel random numbers: as easy as 1, 2, 3"): ten rounds of
  the Philox-4x32 bijection, multipliers 0xD2511F53 and 0xCD9E8D57, key
  increments 0x9E3779B9 and 0xBB67AE85. Random numbers of the sampler come
  from it on both sides (the GPU implements the same published definition);
* ``uniform01`` and ``normal_pair``: a 52-bit uniform in (0, 1) from two words
  and the Box-Muller transform of two uniforms;
* ``draw_theta``: hyperparameters from the training prior (log-uniform);
* ``sample_curve``: the SHO process by its exact discretisation (the matrix
  exponential of the oscillator's drift and the stationary covariance; the
  same state-space form the paper's celerite solvers rest on, Appendix A),
  plus white noise on a unit baseline;
* ``bin_input``: the CNN input (bin means of the flux over 512 equal time
  bins, divided by their median, minus one, times 100; empty bins 0);
* ``cnn_forward`` / ``cnn_backward`` / ``adam_step``: the network (four
  stride-2 convolutions of width 7 with 64 channels and ReLU, global average
  pool, linear head to four outputs), its mean-squared-error gradient and
  one Adam step;
* ``nll_dense`` / ``nll_kalman``: the negative log-likelihood of Eq. 5 for
  the trend-only model with the trend profiled, by the dense Cholesky and by
  the Kalman filter's prediction-error decomposition;
* ``plain_init`` and ``fit_bfgs``: the plain fit that checks the warm start,
  a Lomb-Scargle period with moment estimates, then BFGS (SciPy).

Readings (the paper gives no network or sampler): listed in the design
notes of the repository; the ones that fix numbers here are the Philox
counter layout (sample index, curve index low and high words, stream), the
uniform and Box-Muller forms above, the bin edges (floor of the time
fraction times the bin count, the last sample in the last bin) and the
median over the non-empty bin means.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.optimize
import scipy.signal

MASK32 = 0xFFFFFFFF
PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)

# Philox streams of the sampler (fourth counter word)
STREAM_PROCESS, STREAM_WHITE, STREAM_INITIAL, STREAM_THETA = 0, 1, 2, 3

# Training prior: log-uniform bounds of (amp, P_rot [d], Q, sigma_w)
PRIOR = {"amp": (0.005, 0.03), "prot": (0.3, 2.0), "q": (1.0, 100.0), "sigma_w": (3e-4, 3e-3)}
TARGET_KEYS = ("amp", "prot", "q", "sigma_w")


# ---------------------------------------------------------------------------
# Counter-based random numbers
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    """Philox-4x32 with 10 rounds: four 32-bit counter words, two key words."""
    c = [int(x) & MASK32 for x in ctr]
    k = [int(x) & MASK32 for x in key]
    for r in range(10):
        if r > 0:
            k = [(k[0] + PHILOX_W[0]) & MASK32, (k[1] + PHILOX_W[1]) & MASK32]
        p0 = PHILOX_M[0] * c[0]
        p1 = PHILOX_M[1] * c[2]
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
    return c


def uniform01(a: int, b: int) -> float:
    """Strictly inside (0, 1): the top 26 bits of a and of b form k < 2^52, and
    (k + 1/2) 2^-52 is exact in FP64."""
    return ((a >> 6) * 67108864.0 + (b >> 6) + 0.5) * (1.0 / 4503599627370496.0)


def normal_pair(words):
    """Box-Muller: two standard normals from the four words of one draw."""
    u1 = uniform01(words[0], words[1])
    u2 = uniform01(words[2], words[3])
    r = math.sqrt(-2.0 * math.log(u1))
    return r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2)


def _ctr(n: int, curve: int, stream: int):
    return [n & MASK32, curve & MASK32, (curve >> 32) & MASK32, stream]


def _key(seed: int):
    return [seed & MASK32, (seed >> 32) & MASK32]


def draw_theta(seed: int, curve: int) -> dict:
    """Hyperparameters from the training prior: four log-uniform draws."""
    w = philox4x32_10(_ctr(0, curve, STREAM_THETA), _key(seed)) + \
        philox4x32_10(_ctr(1, curve, STREAM_THETA), _key(seed))
    out = {}
    for i, name in enumerate(TARGET_KEYS):
        lo, hi = PRIOR[name]
        u = uniform01(w[2 * i], w[2 * i + 1])
        out[name] = math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))
    return out


def omega_from_rotation(prot: float, q: float) -> float:
    """SHO frequency whose Q > 1/2 oscillation has period prot (2 pi / prot for Q <= 1/2)."""
    if q > 0.5:
        return 4.0 * math.pi * q / (prot * math.sqrt(4.0 * q * q - 1.0))
    return 2.0 * math.pi / prot


# ---------------------------------------------------------------------------
# GP sampler and CNN input
# ---------------------------------------------------------------------------

def sho_transition(amp: float, omega: float, q: float, h: float):
    """State transition over a step h and the Cholesky factor of its noise:
    Phi = expm(F h), Qd = Pinf - Phi Pinf Phi^T for the drift F of
    x'' + (omega/Q) x' + omega^2 x = white forcing, Pinf = diag(amp^2, amp^2 omega^2)."""
    F = np.array([[0.0, 1.0], [-omega * omega, -omega / q]])
    Pinf = np.diag([amp * amp, amp * amp * omega * omega])
    Phi = scipy.linalg.expm(F * h)
    Qd = Pinf - Phi @ Pinf @ Phi.T
    c00 = math.sqrt(max(Qd[0, 0], 0.0))
    c10 = Qd[1, 0] / c00 if c00 > 0 else 0.0
    c11 = math.sqrt(max(Qd[1, 1] - c10 * c10, 0.0))
    return Phi, np.array([[c00, 0.0], [c10, c11]])


def sample_curve(t: np.ndarray, theta: dict, seed: int, curve: int) -> np.ndarray:
    """f_n = 1 + g(t_n) + sigma_w e_n: g the SHO process (exact discretisation),
    e white; theta = {amp, omega, q, sigma_w}."""
    amp, om, q, sw = theta["amp"], theta["omega"], theta["q"], theta["sigma_w"]
    key = _key(seed)
    n = t.shape[0]
    f = np.empty(n)
    z0, z1 = normal_pair(philox4x32_10(_ctr(0, curve, STREAM_INITIAL), key))
    x = np.array([amp * z0, amp * om * z1])
    cache = {}
    for i in range(n):
        if i > 0:
            h = float(t[i] - t[i - 1])
            if h not in cache:
                cache[h] = sho_transition(amp, om, q, h)
            Phi, C = cache[h]
            za, zb = normal_pair(philox4x32_10(_ctr(i, curve, STREAM_PROCESS), key))
            x = Phi @ x + C @ np.array([za, zb])
        zw, _ = normal_pair(philox4x32_10(_ctr(i, curve, STREAM_WHITE), key))
        f[i] = 1.0 + x[0] + sw * zw
    return f


def bin_index(t: np.ndarray, n_bins: int) -> np.ndarray:
    span = float(t[-1] - t[0])
    b = np.floor((t - t[0]) / span * n_bins).astype(np.int64)
    return np.minimum(b, n_bins - 1)


def bin_input(t: np.ndarray, f: np.ndarray, n_bins: int = 512) -> np.ndarray:
    """100 (m_b / median(m) - 1) over the non-empty bin means m_b; empty bins 0."""
    b = bin_index(t, n_bins)
    s = np.zeros(n_bins)
    c = np.zeros(n_bins)
    for i in range(t.shape[0]):
        s[b[i]] += f[i]
        c[b[i]] += 1
    ok = c > 0
    m = np.where(ok, s / np.where(ok, c, 1), 0.0)
    med = float(np.median(m[ok]))
    return np.where(ok, 100.0 * (m / med - 1.0), 0.0)


def standardise(theta: dict) -> np.ndarray:
    """Targets: logs of (amp, P_rot, Q, sigma_w) centred and scaled by the prior's log-uniform moments."""
    out = []
    for name in TARGET_KEYS:
        lo, hi = PRIOR[name]
        mu = 0.5 * (math.log(lo) + math.log(hi))
        sd = (math.log(hi) - math.log(lo)) / math.sqrt(12.0)
        out.append((math.log(theta[name]) - mu) / sd)
    return np.array(out)


def unstandardise(y) -> dict:
    out = {}
    for i, name in enumerate(TARGET_KEYS):
        lo, hi = PRIOR[name]
        mu = 0.5 * (math.log(lo) + math.log(hi))
        sd = (math.log(hi) - math.log(lo)) / math.sqrt(12.0)
        out[name] = math.exp(mu + sd * float(y[i]))
    return out


# ---------------------------------------------------------------------------
# The network
# ---------------------------------------------------------------------------

KW, STRIDE, PAD, CH, N_OUT = 7, 2, 3, 64, 4
LAYERS = 4


def param_shapes(n_in: int = 1):
    """Flat parameter order: (W1, b1, ..., W4, b4, Wh, bh)."""
    shapes = []
    cin = n_in
    for _ in range(LAYERS):
        shapes += [("W", (CH, cin, KW)), ("b", (CH,))]
        cin = CH
    shapes += [("Wh", (N_OUT, CH)), ("bh", (N_OUT,))]
    return shapes


def unflatten(flat: np.ndarray):
    out, o = [], 0
    for _, shp in param_shapes():
        n = int(np.prod(shp))
        out.append(flat[o:o + n].reshape(shp))
        o += n
    return out


def n_params() -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes())


def conv1d(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """z[b, co, l] = b[co] + sum_ci sum_k W[co, ci, k] x[b, ci, 2 l + k - 3] (zero outside)."""
    B, ci, L = x.shape
    lo = L // STRIDE
    xp = np.zeros((B, ci, L + 2 * PAD))
    xp[:, :, PAD:PAD + L] = x
    z = np.zeros((B, W.shape[0], lo)) + b[None, :, None]
    for k in range(KW):
        cols = xp[:, :, k:k + STRIDE * lo:STRIDE]          # (B, ci, lo)
        z += np.einsum("oc,bcl->bol", W[:, :, k], cols)
    return z


def cnn_forward(flat: np.ndarray, x: np.ndarray):
    """x (B, 512) -> outputs (B, 4) and the activations the backward needs."""
    P = unflatten(flat)
    acts = [x[:, None, :]]
    h = acts[0]
    for i in range(LAYERS):
        h = np.maximum(conv1d(h, P[2 * i], P[2 * i + 1]), 0.0)
        acts.append(h)
    pooled = h.mean(axis=2)
    out = pooled @ P[-2].T + P[-1]
    return out, (acts, pooled)


def mse(out: np.ndarray, y: np.ndarray) -> float:
    return float(np.mean((out - y) ** 2))


def cnn_backward(flat: np.ndarray, x: np.ndarray, y: np.ndarray):
    """Loss and its gradient with respect to the flat parameters."""
    P = unflatten(flat)
    out, (acts, pooled) = cnn_forward(flat, x)
    B = x.shape[0]
    dout = 2.0 * (out - y) / (B * N_OUT)
    grads = [None] * len(P)
    grads[-2] = dout.T @ pooled
    grads[-1] = dout.sum(axis=0)
    dpool = dout @ P[-2]
    L = acts[-1].shape[2]
    dh = np.repeat(dpool[:, :, None], L, axis=2) / L
    for i in reversed(range(LAYERS)):
        dz = dh * (acts[i + 1] > 0)
        xin = acts[i]
        Lin = xin.shape[2]
        lo = dz.shape[2]
        xp = np.zeros((B, xin.shape[1], Lin + 2 * PAD))
        xp[:, :, PAD:PAD + Lin] = xin
        dW = np.zeros_like(P[2 * i])
        dxp = np.zeros_like(xp)
        for k in range(KW):
            cols = xp[:, :, k:k + STRIDE * lo:STRIDE]
            dW[:, :, k] = np.einsum("bol,bcl->oc", dz, cols)
            dxp[:, :, k:k + STRIDE * lo:STRIDE] += np.einsum("oc,bol->bcl", P[2 * i][:, :, k], dz)
        grads[2 * i] = dW
        grads[2 * i + 1] = dz.sum(axis=(0, 2))
        dh = dxp[:, :, PAD:PAD + Lin]
    return mse(out, y), np.concatenate([g.reshape(-1) for g in grads])


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (any fixed draw serves the tests)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in param_shapes():
        if name in ("b", "bh"):
            parts.append(np.zeros(shp))
        else:
            fan_in = int(np.prod(shp[1:]))
            lim = math.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, shp))
    return np.concatenate([p.reshape(-1) for p in parts])


def adam_step(p, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) at step t >= 1; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Likelihood of the trend-only model (Eq. 5) with the trend profiled
# ---------------------------------------------------------------------------

def _profiled(ft: np.ndarray, At: np.ndarray) -> float:
    """chi^2 of the GLS trend fit from whitened flux and trend."""
    if At.shape[1] == 0:
        return float(ft @ ft)
    G = At.T @ At
    w = np.linalg.solve(G, At.T @ ft)
    r = ft - At @ w
    return float(r @ r)


def nll_dense(t, f, A, theta: dict) -> float:
    """-ln L_0 of Eq. 5: chi2_0/2 + ln|K|/2 + (N/2) ln 2 pi, K dense, Cholesky-whitened."""
    from oracle import gp
    K = gp.covariance(np.asarray(t, dtype=np.float64), theta)
    L = gp.cholesky(K)
    ft = scipy.linalg.solve_triangular(L, f, lower=True)
    At = scipy.linalg.solve_triangular(L, A, lower=True) if A.shape[1] else A
    return 0.5 * _profiled(ft, At) + 0.5 * gp.logdet(L) + 0.5 * len(f) * math.log(2.0 * math.pi)


def nll_kalman(t, f, A, theta: dict) -> float:
    """The same likelihood by the Kalman filter of the SHO state-space model:
    innovations e_n with variances S_n whiten every column of [A | f] (the gain
    depends on theta only), and ln|K| = sum ln S_n."""
    amp, om, q, sw = theta["amp"], theta["omega"], theta["q"], theta["sigma_w"]
    Y = np.column_stack([A, f]) if A.shape[1] else f[:, None]
    n, m = Y.shape
    Pinf = np.diag([amp * amp, amp * amp * om * om])
    P = Pinf.copy()
    X = np.zeros((2, m))               # predicted state means, one per column
    W = np.empty((n, m))
    logdet = 0.0
    for i in range(n):
        if i > 0:
            Phi, C = sho_transition(amp, om, q, float(t[i] - t[i - 1]))
            X = Phi @ X
            P = Phi @ P @ Phi.T + C @ C.T
        S = P[0, 0] + sw * sw
        e = Y[i] - X[0]
        W[i] = e / math.sqrt(S)
        logdet += math.log(S)
        Kg = P[:, 0] / S
        X = X + np.outer(Kg, e)
        P = P - np.outer(Kg, P[0, :])
    ft = W[:, -1]
    At = W[:, :-1]
    return 0.5 * _profiled(ft, At) + 0.5 * logdet + 0.5 * n * math.log(2.0 * math.pi)


# ---------------------------------------------------------------------------
# The plain fit (fallback and check)
# ---------------------------------------------------------------------------

def plain_init(t, f, prot_grid) -> dict:
    """Lomb-Scargle peak period (SciPy), amp = std(f), Q = 5,
    sigma_w = rms of second differences / sqrt(6) (white noise dominates them)."""
    t = np.asarray(t, dtype=np.float64)
    y = f - f.mean()
    w = 2.0 * np.pi / np.asarray(prot_grid)
    pw = scipy.signal.lombscargle(t, y, w)
    prot = float(prot_grid[int(np.argmax(pw))])
    d2 = f[2:] - 2.0 * f[1:-1] + f[:-2]
    return {"amp": float(np.std(f)), "prot": prot, "q": 5.0,
            "sigma_w": float(np.sqrt(np.mean(d2 * d2) / 6.0))}


def theta_from_x(x) -> dict:
    """Fit coordinates x = (ln amp, ln P_rot, ln Q, ln sigma_w) -> SHO parameters."""
    amp, prot, q, sw = (math.exp(v) for v in x)
    return {"amp": amp, "omega": omega_from_rotation(prot, q), "q": q, "sigma_w": sw}


def fit_bfgs(t, f, A, start: dict, nll=nll_kalman, gtol=1e-5, maxiter=200):
    """BFGS (SciPy) on the profiled NLL in log coordinates from ``start`` = {amp, prot, q, sigma_w}."""
    x0 = np.log([start["amp"], start["prot"], start["q"], start["sigma_w"]])

    def fun(x):
        try:
            v = nll(t, f, A, theta_from_x(x))
        except (np.linalg.LinAlgError, ValueError, OverflowError):
            return 1e300
        return v if np.isfinite(v) else 1e300

    res = scipy.optimize.minimize(fun, x0, method="BFGS", options={"gtol": gtol, "maxiter": maxiter})
    return res

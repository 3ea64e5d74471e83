"""Linear-prediction (Prony) ringdown fit, written plainly in NumPy FP64.

TEST INFRASTRUCTURE ONLY: used by tests/ to check the library's fit.

The paper extracts the resonance frequency and Q of the CPW resonator from
probe time series with ESPRIT (Sec. 5, Table 7) without giving its settings.
This is the fit the library implements instead: the decimated window
x_m = series[start + m*decim] is modelled by x_m = sum_{k=1}^{P} a_k x_{m-k};
a is the least-squares solution over m = P .. M-1; each root z of
z^P - a_1 z^{P-1} - ... - a_P is a damped mode z = exp((-alpha + i 2 pi f) ts)
with ts = decim dt, and Q = pi f / alpha.  The reported mode is the one of
largest least-squares amplitude within [0.5, 1.5] f_hint.
"""
import numpy as np


def lp_fit(series, start, count, decim, order, dt, f_hint=0.0):
    x = np.asarray(series, dtype=np.float64)[start:start + (count - 1) * decim + 1:decim]
    assert x.size == count
    P = order
    A = np.stack([x[P - k:count - k] for k in range(1, P + 1)], axis=1)
    b = x[P:count]
    a, *_ = np.linalg.lstsq(A, b, rcond=None)
    resid = np.sum((b - A @ a) ** 2) / np.sum(x[P:count] ** 2)
    z = np.roots(np.concatenate([[1.0], -a]))
    ts = decim * dt
    lz = np.log(z.astype(complex))
    f = lz.imag / (2 * np.pi * ts)
    alpha = -lz.real / ts
    # Prony's last step: complex amplitudes of the modes by least squares on the window
    V = z[None, :] ** np.arange(count)[:, None]
    c, *_ = np.linalg.lstsq(V, x.astype(complex), rcond=None)
    amp = np.abs(c)
    pos = np.where(f > 0)[0]
    near = pos[(f[pos] >= 0.5 * f_hint) & (f[pos] <= 1.5 * f_hint)] if f_hint > 0 else pos
    cand = near if len(near) else pos
    i = cand[np.argmax(amp[cand])]
    return dict(f0=f[i], alpha=alpha[i], Q=np.pi * f[i] / alpha[i], residual=resid, modes=list(zip(f, alpha)),
                amplitudes=amp)

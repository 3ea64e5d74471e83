"""ESPRIT estimate of resonance frequencies and damping from a ringdown, in NumPy FP64.

TEST INFRASTRUCTURE ONLY: used by tests/ to check the library's ESPRIT fit.

The paper extracts the resonance frequency and quality factor of its CPW
resonator from probe time series with ESPRIT (Sec. 5, Table 7) and gives no
settings.  This is the textbook least-squares ESPRIT (estimation of signal
parameters via rotational invariance, Roy and Kailath 1989) applied to a sum
of damped complex exponentials x_m = sum_q c_q z_q^m:

  1. the decimated window x_m = series[start + m*decim], m = 0 .. count-1, is
     arranged in the Hankel matrix H[r, j] = x_{r+j} with `pencil` columns and
     count - pencil + 1 rows;
  2. the p right singular vectors of H with the largest singular values span
     the signal subspace V_s (pencil x p);
  3. with V_1 = V_s without its last row and V_2 = V_s without its first, the
     shift invariance V_2 = V_1 Phi is solved by least squares;
  4. the eigenvalues of Phi are the modes z_q = exp((-alpha_q + i 2 pi f_q) ts),
     ts = decim dt; Q = pi f / alpha;
  5. the complex amplitudes c_q follow from least squares on the window
     (Vandermonde system), and the reported mode is the largest-amplitude one
     with f in [0.5, 1.5] f_hint (the largest-amplitude one with f > 0 if
     f_hint <= 0 or none lies there).

A real damped cosine contributes the conjugate pair z, conj(z): p = 2 per mode.
"""
import numpy as np


def hankel(x, pencil):
    L = x.size - pencil + 1
    return np.stack([x[j:j + L] for j in range(pencil)], axis=1)


def esprit(series, start, count, decim, order, dt, pencil, f_hint=0.0):
    x = np.asarray(series, dtype=np.float64)[start:start + (count - 1) * decim + 1:decim]
    assert x.size == count and 2 <= order < pencil <= count // 2
    H = hankel(x, pencil)
    _, s, Vh = np.linalg.svd(H, full_matrices=False)
    Vs = Vh[:order].conj().T
    Phi, *_ = np.linalg.lstsq(Vs[:-1], Vs[1:], rcond=None)
    z = np.linalg.eigvals(Phi)
    ts = decim * dt
    lz = np.log(z.astype(complex))
    f = lz.imag / (2 * np.pi * ts)
    alpha = -lz.real / ts
    Vm = z[None, :] ** np.arange(count)[:, None]
    c, *_ = np.linalg.lstsq(Vm, x.astype(complex), rcond=None)
    amp = np.abs(c)
    pos = np.where(f > 0)[0]
    near = pos[(f[pos] >= 0.5 * f_hint) & (f[pos] <= 1.5 * f_hint)] if f_hint > 0 else pos
    cand = near if len(near) else pos
    i = cand[np.argmax(amp[cand])]
    sv2 = s ** 2
    return dict(f0=f[i], alpha=alpha[i], Q=np.pi * f[i] / alpha[i], modes=list(zip(f, alpha)), amplitudes=amp,
                residual=float(sv2[order:].sum() / sv2.sum()))

// C ABI of the ringdown fit: GPU normal equations, host P x P solve and roots.
#include <cmath>
#include <complex>
#include <vector>

#include "sim_internal.h"

using namespace tfl;
using namespace tfl::detail;

namespace {

using cplx = std::complex<double>;

// Minimum-norm solution of the symmetric positive semi-definite system A a = r
// (n x n, row major): cyclic Jacobi eigen-decomposition A = V diag(w) V^T,
// a = V diag(1/w) V^T r over the eigenvalues above 1e-13 max(w).
bool solve(std::vector<double> A, const std::vector<double> &r, int n, std::vector<double> &a,
           std::vector<double> *eig = nullptr)
{
    std::vector<double> V(n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += A[i * n + i] * A[i * n + i];
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        }
        if (!(off > 1e-30 * diag)) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {  // A <- J^T A J
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - sn * akq;
                    A[k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - sn * aqk;
                    A[q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - sn * vkq;
                    V[k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    double wmax = 0.0;
    for (int i = 0; i < n; ++i) wmax = std::max(wmax, A[i * n + i]);
    if (eig) {
        eig->resize(n);
        for (int i = 0; i < n; ++i) (*eig)[i] = A[i * n + i];
    }
    if (!(wmax > 0.0) || !std::isfinite(wmax)) return false;
    a.assign(n, 0.0);
    for (int e = 0; e < n; ++e) {
        const double w = A[e * n + e];
        if (!(w > 1e-13 * wmax)) continue;
        double proj = 0.0;
        for (int k = 0; k < n; ++k) proj += V[k * n + e] * r[k];
        for (int k = 0; k < n; ++k) a[k] += V[k * n + e] * proj / w;
    }
    return true;
}

// Roots of the monic polynomial z^n + c[1] z^{n-1} + ... + c[n] (Durand-Kerner
// simultaneous iteration, then Newton polishing).
bool poly_roots(const std::vector<double> &c, int n, std::vector<cplx> &z)
{
    auto p = [&](cplx x) {
        cplx v = 1.0;
        for (int q = 1; q <= n; ++q) v = v * x + c[q];
        return v;
    };
    auto dp = [&](cplx x) {
        cplx v = 0.0, w = 1.0;
        for (int q = 1; q <= n; ++q) {
            v = v * x + w;
            w = w * x + c[q];
        }
        return v;
    };
    double bound = 0.0;
    for (int q = 1; q <= n; ++q) bound = std::max(bound, std::pow(std::fabs(c[q]), 1.0 / q));
    bound = 2.0 * std::max(bound, 1e-3);
    z.resize(n);
    const cplx seed(0.4, 0.9);
    for (int i = 0; i < n; ++i) z[i] = bound * std::pow(seed, i) / std::abs(std::pow(seed, i));
    bool conv = false;
    for (int it = 0; it < 2000 && !conv; ++it) {
        double dmax = 0.0;
        for (int i = 0; i < n; ++i) {
            cplx den = 1.0;
            for (int j = 0; j < n; ++j)
                if (j != i) den *= (z[i] - z[j]);
            const cplx d = p(z[i]) / den;
            z[i] -= d;
            dmax = std::max(dmax, std::abs(d) / std::max(std::abs(z[i]), 1e-300));
        }
        conv = dmax < 1e-15;
    }
    for (int i = 0; i < n; ++i)
        for (int it = 0; it < 3; ++it) {
            const cplx d = dp(z[i]);
            if (std::abs(d) > 0.0) z[i] -= p(z[i]) / d;
        }
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(z[i].real()) || !std::isfinite(z[i].imag())) return false;
    return true;
}

int fit_order(tfl_sim *s, const double *series, const tfl_fit_req *rq, int P, tfl_fit_result *out, hipStream_t st)
{
    const int npairs = (P + 1) * (P + 2) / 2;
    double *dev = s->scratch;  // pairs fit in the reduction region
    hipError_t e = launch_gram(series, rq->start, rq->count, rq->decim, P, dev, st);
    if (e != hipSuccess) return hip_fail(s, e, "gram");
    std::vector<double> g(npairs);
    e = hipMemcpyAsync(g.data(), dev, npairs * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(s, e, "gram readback");
    auto G = [&](int j, int k) {
        if (j > k) std::swap(j, k);
        const int row = j * (P + 1) - j * (j - 1) / 2;  // start of row j in the packed upper triangle
        return g[row + (k - j)];
    };
    std::vector<double> A(P * P), r(P), a;
    for (int j = 1; j <= P; ++j) {
        r[j - 1] = G(0, j);
        for (int k = 1; k <= P; ++k) A[(j - 1) * P + (k - 1)] = G(j, k);
    }
    if (!solve(A, r, P, a)) return fail(s, TFL_E_NONFINITE, "singular normal equations (order %d)", P);
    // two steps of iterative refinement with the correction formed from the data on the device
    double *dev_a = s->scratch + 512, *dev_r = s->scratch + 1024;
    for (int it = 0; it < 2; ++it) {
        std::vector<double> corr(P), da;
        e = hipMemcpyAsync(dev_a, a.data(), P * sizeof(double), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = launch_lp_residual(series, rq->start, rq->count, rq->decim, P, dev_a, dev_r, st);
        if (e == hipSuccess) e = hipMemcpyAsync(corr.data(), dev_r, P * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(s, e, "lp refinement");
        if (!solve(A, corr, P, da)) break;
        for (int q = 0; q < P; ++q) a[q] += da[q];
    }
    double res = G(0, 0);
    for (int j = 1; j <= P; ++j) {
        res -= 2.0 * a[j - 1] * G(0, j);
        for (int k = 1; k <= P; ++k) res += a[j - 1] * a[k - 1] * G(j, k);
    }
    std::vector<double> c(P + 1);
    c[0] = 1.0;
    for (int q = 1; q <= P; ++q) c[q] = -a[q - 1];
    std::vector<cplx> z;
    if (!poly_roots(c, P, z)) return fail(s, TFL_E_NONFINITE, "root iteration failed (order %d)", P);
    const double ts = (double)rq->decim * s->cfg.dt;
    out->order = P;
    out->nmodes = P;
    out->residual = G(0, 0) > 0.0 ? std::max(res, 0.0) / G(0, 0) : 0.0;
    // mode amplitudes: least squares x_m = sum_q c_q z_q^m over the window (Prony's last step)
    std::vector<double> amp(P, 0.0);
    {
        const long long M = rq->count;
        std::vector<double> win((size_t)((M - 1) * rq->decim + 1));
        e = hipMemcpyAsync(win.data(), series + rq->start, win.size() * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(s, e, "fit window readback");
        std::vector<cplx> N(P * P, 0.0), rhs(P, 0.0), pw(P, 1.0);
        for (long long m = 0; m < M; ++m) {
            const double xm = win[(size_t)(m * rq->decim)];
            for (int q = 0; q < P; ++q) {
                rhs[q] += std::conj(pw[q]) * xm;
                for (int t = 0; t < P; ++t) N[q * P + t] += std::conj(pw[q]) * pw[t];
            }
            for (int q = 0; q < P; ++q) pw[q] *= z[q];
        }
        // complex Gaussian elimination with partial pivoting
        bool ok = true;
        for (int c = 0; c < P && ok; ++c) {
            int pv = c;
            for (int i = c + 1; i < P; ++i)
                if (std::abs(N[i * P + c]) > std::abs(N[pv * P + c])) pv = i;
            if (!(std::abs(N[pv * P + c]) > 0.0)) { ok = false; break; }
            if (pv != c) {
                for (int q = 0; q < P; ++q) std::swap(N[c * P + q], N[pv * P + q]);
                std::swap(rhs[c], rhs[pv]);
            }
            for (int i = c + 1; i < P; ++i) {
                const cplx f = N[i * P + c] / N[c * P + c];
                for (int q = c; q < P; ++q) N[i * P + q] -= f * N[c * P + q];
                rhs[i] -= f * rhs[c];
            }
        }
        if (ok) {
            std::vector<cplx> cq(P);
            for (int i = P - 1; i >= 0; --i) {
                cplx v = rhs[i];
                for (int q = i + 1; q < P; ++q) v -= N[i * P + q] * cq[q];
                cq[i] = v / N[i * P + i];
            }
            for (int q = 0; q < P; ++q) amp[q] = std::isfinite(std::abs(cq[q])) ? std::abs(cq[q]) : 0.0;
        }
    }
    // report: the largest-amplitude mode with f in [0.5, 1.5] f_hint (f_hint > 0), else the
    // largest-amplitude mode with f > 0
    int best = -1;
    for (int pass = 0; pass < 2 && best < 0; ++pass)
        for (int q = 0; q < P; ++q) {
            const cplx lz = std::log(z[q]);
            const double f = lz.imag() / (kTwoPi * ts), al = -lz.real() / ts;
            out->modes[2 * q] = f;
            out->modes[2 * q + 1] = al;
            if (!(f > 0.0)) continue;
            if (pass == 0 && rq->f_hint > 0.0 && (f < 0.5 * rq->f_hint || f > 1.5 * rq->f_hint)) continue;
            if (best < 0 || amp[q] > amp[best]) best = q;
        }
    if (best < 0) return fail(s, TFL_E_NONFINITE, "no mode with positive frequency");
    out->f0 = out->modes[2 * best];
    out->alpha = out->modes[2 * best + 1];
    out->Q = kTwoPi / 2.0 * out->f0 / out->alpha;
    return TFL_OK;
}

}  // namespace

// Model order from the data: the number of eigenvalues of the order-16
// Gram matrix of the lagged samples above 1e-8 of the largest (components whose
// amplitude is at least ~1e-4 of the dominant one), at least 2.
int auto_order(tfl_sim *s, const double *series, const tfl_fit_req *rq, hipStream_t st, int *P)
{
    const int Pm = TFL_FIT_MAX_ORDER;
    const int npairs = (Pm + 1) * (Pm + 2) / 2;
    hipError_t e = launch_gram(series, rq->start, rq->count, rq->decim, Pm, s->scratch, st);
    std::vector<double> g(npairs);
    if (e == hipSuccess) e = hipMemcpyAsync(g.data(), s->scratch, npairs * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(s, e, "gram (order selection)");
    std::vector<double> A(Pm * Pm), r(Pm, 0.0), a, w;
    for (int j = 1; j <= Pm; ++j)
        for (int k = 1; k <= Pm; ++k) {
            int jj = j, kk = k;
            if (jj > kk) std::swap(jj, kk);
            A[(j - 1) * Pm + (k - 1)] = g[jj * (Pm + 1) - jj * (jj - 1) / 2 + (kk - jj)];
        }
    if (!solve(A, r, Pm, a, &w)) return fail(s, TFL_E_NONFINITE, "singular Gram matrix (order selection)");
    double wmax = 0.0;
    for (double v : w) wmax = std::max(wmax, v);
    int rank = 0;
    for (double v : w) rank += (v > 1e-8 * wmax) ? 1 : 0;
    *P = std::max(2, std::min(Pm, rank));
    return TFL_OK;
}

extern "C" int tfl_ringdown_fit(tfl_sim *s, int probe_id, const tfl_fit_req *rq, tfl_fit_result *out, void *stream)
{
    int rc = check_bound(s, false);
    if (rc != TFL_OK) return rc;
    if (!rq || !out) return fail(s, TFL_E_INVAL, "null argument");
    if (probe_id < 0 || probe_id >= (int)s->probe.size()) return fail(s, TFL_E_INVAL, "bad probe id");
    const ProbeDesc &p = s->probe[probe_id];
    if (!p.series) return fail(s, TFL_E_INVAL, "probe has no series buffer");
    if (rq->order < 0 || rq->order > TFL_FIT_MAX_ORDER)
        return fail(s, TFL_E_INVAL, "order must be 0..%d", TFL_FIT_MAX_ORDER);
    if (rq->decim < 1 || rq->start < 0 || rq->count <= 2 * TFL_FIT_MAX_ORDER ||
        rq->start + (rq->count - 1) * rq->decim >= p.cap)
        return fail(s, TFL_E_INVAL, "fit window outside the probe series or too short");
    hipStream_t st = (hipStream_t)stream;
    *out = tfl_fit_result{};
    int P = rq->order;
    if (P == 0 && (rc = auto_order(s, p.series, rq, st, &P)) != TFL_OK) return rc;
    return fit_order(s, p.series, rq, P, out, st);
}

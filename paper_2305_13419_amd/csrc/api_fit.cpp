// C ABI of the ringdown fit: GPU normal equations, host P x P solve and roots.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "sim_internal.h"

using namespace tfl;
using namespace tfl::detail;

namespace {

using cplx = std::complex<double>;

// Cyclic Jacobi eigen-decomposition of the symmetric n x n matrix A (row major):
// A = V diag(w) V^T, eigenvector e in column e of V.
void jacobi_eig(std::vector<double> A, int n, std::vector<double> &w, std::vector<double> &V)
{
    V.assign((size_t)n * n, 0.0);
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
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

// Minimum-norm solution of the symmetric positive semi-definite system A a = r
// (n x n, row major): a = V diag(1/w) V^T r over the eigenvalues above 1e-13 max(w).
bool solve(const std::vector<double> &A, const std::vector<double> &r, int n, std::vector<double> &a,
           std::vector<double> *eig = nullptr)
{
    std::vector<double> w, V;
    jacobi_eig(A, n, w, V);
    double wmax = 0.0;
    for (int i = 0; i < n; ++i) wmax = std::max(wmax, w[i]);
    if (eig) *eig = w;
    if (!(wmax > 0.0) || !std::isfinite(wmax)) return false;
    a.assign(n, 0.0);
    for (int e = 0; e < n; ++e) {
        if (!(w[e] > 1e-13 * wmax)) continue;
        double proj = 0.0;
        for (int k = 0; k < n; ++k) proj += V[k * n + e] * r[k];
        for (int k = 0; k < n; ++k) a[k] += V[k * n + e] * proj / w[e];
    }
    return true;
}

// Eigenvalues of the real n x n matrix A (row major): Householder reduction to
// upper Hessenberg form, then single-shift QR iterations in complex arithmetic
// with Wilkinson shifts and deflation on negligible subdiagonal entries.
bool eig_general(const std::vector<double> &A, int n, std::vector<cplx> &ev)
{
    std::vector<cplx> H((size_t)n * n);
    for (int i = 0; i < n * n; ++i) H[i] = A[i];
    auto h = [&](int i, int j) -> cplx & { return H[(size_t)i * n + j]; };
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        std::vector<cplx> v(m);
        double xn = 0.0;
        for (int i = 0; i < m; ++i) {
            v[i] = h(k + 1 + i, k);
            xn += std::norm(v[i]);
        }
        xn = std::sqrt(xn);
        if (!(xn > 0.0)) continue;
        const cplx alpha = -std::polar(xn, std::arg(v[0]));
        v[0] -= alpha;
        double vn = 0.0;
        for (int i = 0; i < m; ++i) vn += std::norm(v[i]);
        if (!(vn > 0.0)) continue;
        for (int j = 0; j < n; ++j) {  // rows k+1.. : (I - 2 v v^H / v^H v) H
            cplx sdot = 0.0;
            for (int i = 0; i < m; ++i) sdot += std::conj(v[i]) * h(k + 1 + i, j);
            const cplx f = 2.0 * sdot / vn;
            for (int i = 0; i < m; ++i) h(k + 1 + i, j) -= f * v[i];
        }
        for (int i = 0; i < n; ++i) {  // columns k+1.. : H (I - 2 v v^H / v^H v)
            cplx sdot = 0.0;
            for (int j = 0; j < m; ++j) sdot += h(i, k + 1 + j) * v[j];
            const cplx f = 2.0 * sdot / vn;
            for (int j = 0; j < m; ++j) h(i, k + 1 + j) -= f * std::conj(v[j]);
        }
    }
    ev.assign(n, 0.0);
    int hi = n - 1, iter = 0;
    std::vector<cplx> rc(n), rs(n);
    while (hi >= 0) {
        if (hi == 0) {
            ev[0] = h(0, 0);
            break;
        }
        int l = hi;
        for (; l > 0; --l) {
            const double sc = std::abs(h(l - 1, l - 1)) + std::abs(h(l, l));
            if (std::abs(h(l, l - 1)) <= 1e-15 * (sc > 0.0 ? sc : 1.0)) {
                h(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == hi) {
            ev[hi] = h(hi, hi);
            --hi;
            iter = 0;
            continue;
        }
        if (++iter > 500) return false;
        const cplx a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
        const cplx half = 0.5 * (a + d), disc = std::sqrt(half * half - (a * d - b * c));
        cplx mu = (std::abs(half + disc - d) < std::abs(half - disc - d)) ? half + disc : half - disc;
        if (iter % 16 == 15) mu = d + 0.75 * std::abs(c);  // exceptional shift
        for (int k = l; k <= hi; ++k) h(k, k) -= mu;
        for (int k = l; k < hi; ++k) {  // H - mu I = Q R by Givens rotations on rows k, k+1
            const cplx x = h(k, k), y = h(k + 1, k);
            const double r = std::sqrt(std::norm(x) + std::norm(y));
            const cplx cc = r > 0.0 ? x / r : cplx(1.0), ss = r > 0.0 ? y / r : cplx(0.0);
            for (int j = k; j <= hi; ++j) {
                const cplx h1 = h(k, j), h2 = h(k + 1, j);
                h(k, j) = std::conj(cc) * h1 + std::conj(ss) * h2;
                h(k + 1, j) = -ss * h1 + cc * h2;
            }
            rc[k] = cc;
            rs[k] = ss;
        }
        for (int k = l; k < hi; ++k) {  // R Q + mu I
            for (int i = l; i <= std::min(k + 2, hi); ++i) {
                const cplx h1 = h(i, k), h2 = h(i, k + 1);
                h(i, k) = h1 * rc[k] + h2 * rs[k];
                h(i, k + 1) = -h1 * std::conj(rs[k]) + h2 * std::conj(rc[k]);
            }
        }
        for (int k = l; k <= hi; ++k) h(k, k) += mu;
    }
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(ev[i].real()) || !std::isfinite(ev[i].imag())) return false;
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

// Prony's last step and the report, shared by both fits: the modes' complex
// amplitudes by least squares x_m = sum_q c_q z_q^m over the window, then the
// largest-amplitude mode with f in [0.5, 1.5] f_hint (f_hint > 0), else the
// largest-amplitude mode with f > 0.  Fills modes, f0, alpha and Q of `out`.
int report_modes(tfl_sim *s, const double *series, const tfl_fit_req *rq, const std::vector<cplx> &z,
                 tfl_fit_result *out, hipStream_t st)
{
    const int P = (int)z.size();
    const double ts = (double)rq->decim * s->cfg.dt;
    hipError_t e;
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
    out->order = P;
    out->nmodes = P;
    out->residual = G(0, 0) > 0.0 ? std::max(res, 0.0) / G(0, 0) : 0.0;
    return report_modes(s, series, rq, z, out, st);
}

// ESPRIT from the pencil Gram matrix.  The device forms G[j][k] = sum_m
// x_{m-j} x_{m-k} (m = M-1 .. count-1) for the M = pencil lags, which is H^T H
// of the Hankel matrix H[r][a] = x_{r+a} with its columns in reverse order;
// its eigenvectors are the right singular vectors of H.  The p leading ones
// span the signal subspace V_s; Phi solves V_s[1:M] = V_s[0:M-1] Phi in the
// least-squares sense and its eigenvalues are the modes z_q.
int esprit_order(tfl_sim *s, const double *series, const tfl_fit_req *rq, int M, tfl_fit_result *out, hipStream_t st)
{
    const int npairs = M * (M + 1) / 2;
    hipError_t e = launch_gram(series, rq->start, rq->count, rq->decim, M - 1, s->scratch, st);
    std::vector<double> g(npairs);
    if (e == hipSuccess) e = hipMemcpyAsync(g.data(), s->scratch, npairs * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(s, e, "pencil gram");
    auto G = [&](int j, int k) {
        if (j > k) std::swap(j, k);
        return g[j * M - j * (j - 1) / 2 + (k - j)];
    };
    std::vector<double> A((size_t)M * M), w, V;
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) A[a * M + b] = G(M - 1 - a, M - 1 - b);
    jacobi_eig(A, M, w, V);
    std::vector<int> idx(M);
    for (int i = 0; i < M; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return w[a] > w[b]; });
    const double wmax = w[idx[0]];
    if (!(wmax > 0.0) || !std::isfinite(wmax)) return fail(s, TFL_E_NONFINITE, "singular pencil Gram matrix");
    int P = rq->order;
    if (P == 0) {
        int rank = 0;
        for (double v : w) rank += (v > 1e-8 * wmax) ? 1 : 0;
        P = std::max(2, std::min(std::min(TFL_FIT_MAX_ORDER, M - 1), rank));
    }
    double tot = 0.0, sig = 0.0;
    for (int i = 0; i < M; ++i) tot += std::max(w[i], 0.0);
    for (int i = 0; i < P; ++i) sig += std::max(w[idx[i]], 0.0);
    // normal equations of the shift invariance: (V1^T V1) Phi = V1^T V2
    auto vs = [&](int row, int col) { return V[(size_t)row * M + idx[col]]; };
    std::vector<double> N((size_t)P * P, 0.0), Phi((size_t)P * P, 0.0);
    for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) {
            double acc = 0.0;
            for (int r = 0; r + 1 < M; ++r) acc += vs(r, a) * vs(r, b);
            N[a * P + b] = acc;
        }
    for (int b = 0; b < P; ++b) {
        std::vector<double> rhs(P), col;
        for (int a = 0; a < P; ++a) {
            double acc = 0.0;
            for (int r = 0; r + 1 < M; ++r) acc += vs(r, a) * vs(r + 1, b);
            rhs[a] = acc;
        }
        if (!solve(N, rhs, P, col)) return fail(s, TFL_E_NONFINITE, "singular shift-invariance equations");
        for (int a = 0; a < P; ++a) Phi[a * P + b] = col[a];
    }
    std::vector<cplx> z;
    if (!eig_general(Phi, P, z)) return fail(s, TFL_E_NONFINITE, "eigenvalue iteration failed (order %d)", P);
    out->order = P;
    out->nmodes = P;
    out->residual = tot > 0.0 ? std::max(tot - sig, 0.0) / tot : 0.0;
    return report_modes(s, series, rq, z, out, st);
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

extern "C" int tfl_esprit_fit(tfl_sim *s, int probe_id, const tfl_fit_req *rq, int32_t pencil, tfl_fit_result *out,
                              void *stream)
{
    int rc = check_bound(s, false);
    if (rc != TFL_OK) return rc;
    if (!rq || !out) return fail(s, TFL_E_INVAL, "null argument");
    if (probe_id < 0 || probe_id >= (int)s->probe.size()) return fail(s, TFL_E_INVAL, "bad probe id");
    const ProbeDesc &p = s->probe[probe_id];
    if (!p.series) return fail(s, TFL_E_INVAL, "probe has no series buffer");
    if (rq->decim < 1 || rq->start < 0 || rq->count < 4 || rq->start + (rq->count - 1) * rq->decim >= p.cap)
        return fail(s, TFL_E_INVAL, "fit window outside the probe series or too short");
    int M = pencil;
    if (M == 0) M = (int)std::min<long long>(TFL_ESPRIT_MAX_PENCIL, rq->count / 3);
    if (M < 3 || M > TFL_ESPRIT_MAX_PENCIL || 2LL * M > rq->count)
        return fail(s, TFL_E_INVAL, "pencil must be in [3, %d] and at most count / 2", TFL_ESPRIT_MAX_PENCIL);
    if (rq->order < 0 || rq->order > TFL_FIT_MAX_ORDER || rq->order >= M)
        return fail(s, TFL_E_INVAL, "order must be 0..min(%d, pencil - 1)", TFL_FIT_MAX_ORDER);
    *out = tfl_fit_result{};
    return esprit_order(s, p.series, rq, M, out, (hipStream_t)stream);
}

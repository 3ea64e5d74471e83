// Reverse-mode (adjoint) sweeps of the two-fluid FDTD step for gfx950.
//
// One forward step is F2 o F1 with
//   F1 (H pass): psiH' = bh psiH + ch D E;  H' = H - dt/mu0 (kh D E + psiH')
//   F2 (E pass): Js' = Js + j E;  psiE' = bn psiE + cn D* H';
//                E' = a E + b (curl_psi H' - Js')            (0 on PEC-wall edges)
// (Algorithm 1 with the half steps fused, Sec. 3).  The adjoint step is
// F1^T o F2^T, evaluated as two sweeps that mirror the forward passes:
//   face sweep: lH += curl(W) with W = b lE (+ the E-side PML transposes)
//               and the H-side PML adjoint variables;
//   edge sweep: lE += -dt/mu0 curl^T lH (+ H-side PML transposes), the
//               objective source, then the edge-local part of F2^T for the
//               preceding step (mu = b lE, lJ, gradient accumulation,
//               lE <- a lE + j lJ).
// Gradients with respect to the per-edge j = dt ell/mu0 and sigma follow from
// dJs'/d ell = dt E/mu0 and dE'/d sigma = -b (theta E'_pre + (1-theta) E).
// The multiplication of a PML adjoint variable by its decay b is applied when
// the variable is next read, so each sweep writes its variables once.
#include "fdtd_common.h"

namespace tfl {
namespace {

// curl term signs: component c differentiated along axis a enters with +1 when
// a = c+1 (mod 3) and -1 when a = c+2 (mod 3), for both curls.
__device__ __forceinline__ int curl_sign(int c, int a) { return ((c + 1) % 3 == a) ? 1 : -1; }
// compact PML array of axis a that holds component c
__device__ __forceinline__ int psi_slot(int c, int a) { return ((c - a + 3) % 3) - 1; }

template <typename T>
__device__ __forceinline__ long long psi_index(const PmlAxis<T> &P, int a, int nx, int ny, int i, int j, int k, int s)
{
    if (a == 0) return ((long long)k * ny + j) * P.P + s;
    if (a == 1) return ((long long)k * P.P + s) * nx + i;
    return ((long long)s * ny + j) * nx + i;
}

// W of an E-side term (edge component c, axis a) at edge (i,j,k): the adjoint of
// the stretched backward difference, sg kn mu + cn tot.
template <typename T>
__device__ __forceinline__ T w_edge(const AdjArgs<T> &A, int c, int a, int i, int j, int k, T muv)
{
    const PmlAxis<T> &P = A.f.pml[a];
    const T sg = T(curl_sign(c, a));
    if (!P.on) return sg * muv;
    const int pos = a == 0 ? i : (a == 1 ? j : k);
    const int s = slab_slot(pos, P.lo, P.hi, P.n);
    if (s < 0) return sg * muv;
    const T tot = A.lpsiE[a][psi_slot(c, a)][psi_index(P, a, A.f.g.nx, A.f.g.ny, i, j, k, s)];
    return sg * P.kn[pos] * muv + P.cn[pos] * tot;
}

// WH of an H-side term (face component h, axis a) at face (i,j,k): the adjoint
// of the stretched forward difference, -dt/mu0 sg kh lH + ch tot.
template <typename T>
__device__ __forceinline__ T w_face(const AdjArgs<T> &A, int h, int a, int i, int j, int k, T lh)
{
    const PmlAxis<T> &P = A.f.pml[a];
    const T sg = T(curl_sign(h, a));
    const T hdt = A.f.hdt;
    if (!P.on) return -hdt * sg * lh;
    const int pos = a == 0 ? i : (a == 1 ? j : k);
    const int s = slab_slot(pos, P.lo, P.hi, P.n);
    if (s < 0) return -hdt * sg * lh;
    const T tot = A.lpsiH[a][psi_slot(h, a)][psi_index(P, a, A.f.g.nx, A.f.g.ny, i, j, k, s)];
    return -hdt * sg * P.kh[pos] * lh + P.ch[pos] * tot;
}

// ---------------------------------------------------------------------------
// Face sweep: lH'' = lH + curl W (F2^T), then the H-side PML variables (F1^T)
// ---------------------------------------------------------------------------
template <typename T, int TY, int TZ>
__global__ __launch_bounds__(kTileX *TY) void adj_face_kernel(const AdjArgs<T> A)
{
    const int nx = A.f.g.nx, ny = A.f.g.ny, nz = A.f.g.nz;
    int i, j, k0, k1;
    if (!tile_of<TY, TZ>(nx, ny, nz, i, j, k0, k1)) return;
    const long long sxy = A.f.g.sxy;
    const int ip = (i + 1 == nx) ? 0 : i + 1;
    const int jp = (j + 1 == ny) ? 0 : j + 1;
    const uint32_t o00 = uint32_t(j * nx + i) * sizeof(T), oxp = uint32_t(j * nx + ip) * sizeof(T);
    const uint32_t oyp = uint32_t(jp * nx + i) * sizeof(T);
    const T rdx = A.f.rd[0], rdy = A.f.rd[1], rdz = A.f.rd[2];
    const T *mx = A.mu[0], *my = A.mu[1], *mz = A.mu[2];
    // the z terms W(Ey, z) and W(Ex, z) of plane k are those of plane k+1 one iteration earlier
    T wyz0, wxz0;
    {
        const long long b = (long long)k0 * sxy;
        wyz0 = w_edge(A, 1, 2, i, j, k0, ldp(my + b, o00));
        wxz0 = w_edge(A, 0, 2, i, j, k0, ldp(mx + b, o00));
    }
    for (int k = k0; k < k1; ++k) {
        const int kp = (k + 1 == nz) ? 0 : k + 1;
        const long long b = opaque_offset((long long)k * sxy), bp = opaque_offset((long long)kp * sxy);
        const T mx0 = ldp(mx + b, o00), my0 = ldp(my + b, o00), mz0 = ldp(mz + b, o00);
        const T my_kp = ldp(my + bp, o00), mx_kp = ldp(mx + bp, o00);
        const T mz_yp = ldp(mz + b, oyp), mz_xp = ldp(mz + b, oxp), mx_yp = ldp(mx + b, oyp), my_xp = ldp(my + b, oxp);
        const T lh0 = ldp(A.lH[0] + b, o00), lh1 = ldp(A.lH[1] + b, o00), lh2 = ldp(A.lH[2] + b, o00);
        // lHx: terms (Ey, z) and (Ez, y)
        const T wyz1 = w_edge(A, 1, 2, i, j, kp, my_kp);
        const T wzy0 = w_edge(A, 2, 1, i, j, k, mz0), wzy1 = w_edge(A, 2, 1, i, jp, k, mz_yp);
        // lHy: terms (Ex, z) and (Ez, x)
        const T wxz1 = w_edge(A, 0, 2, i, j, kp, mx_kp);
        const T wzx0 = w_edge(A, 2, 0, i, j, k, mz0), wzx1 = w_edge(A, 2, 0, ip, j, k, mz_xp);
        // lHz: terms (Ex, y) and (Ey, x)
        const T wxy0 = w_edge(A, 0, 1, i, j, k, mx0), wxy1 = w_edge(A, 0, 1, i, jp, k, mx_yp);
        const T wyx0 = w_edge(A, 1, 0, i, j, k, my0), wyx1 = w_edge(A, 1, 0, ip, j, k, my_xp);
        const T lh[3] = {lh0 + (wyz0 - wyz1) * rdz + (wzy0 - wzy1) * rdy,
                         lh1 + (wxz0 - wxz1) * rdz + (wzx0 - wzx1) * rdx,
                         lh2 + (wxy0 - wxy1) * rdy + (wyx0 - wyx1) * rdx};
        for (int h = 0; h < 3; ++h) stp(A.lH[h] + b, o00, lh[h]);
        wyz0 = wyz1;
        wxz0 = wxz1;
        // H-side PML adjoint variables: tot = bh * stored + (-dt/mu0) sg lH''
        const int pos[3] = {i, j, k};
        for (int a = 0; a < 3; ++a) {
            const PmlAxis<T> &P = A.f.pml[a];
            if (!P.on) continue;
            const int s = slab_slot(pos[a], P.lo, P.hi, P.n);
            if (s < 0) continue;
            const long long pi = psi_index(P, a, nx, ny, i, j, k, s);
            for (int q = 0; q < 2; ++q) {
                const int h = (a + 1 + q) % 3;
                T *ps = A.lpsiH[a][q];
                ps[pi] = P.bh[pos[a]] * ps[pi] - A.f.hdt * T(curl_sign(h, a)) * lh[h];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Edge sweep: lE += curl^T WH (F1^T), objective source, then the edge-local
// part of F2^T of the preceding step with the gradient accumulation.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void edge_cells(const StepArgs<T> &f, int comp, int i, int j, int k, T e[4], T s[4],
                                           T l[4])
{
    const int nx = f.g.nx, ny = f.g.ny, nz = f.g.nz;
    const int im = (i == 0) ? nx - 1 : i - 1;
    const int jm = (j == 0) ? ny - 1 : j - 1;
    const int km = (k == 0) ? nz - 1 : k - 1;
    auto id = [&](int ii, int jj, int kk) { return ((long long)kk * ny + jj) * nx + ii; };
    long long q[4];
    if (comp == 0) { q[0] = id(i, j, k); q[1] = id(i, j, km); q[2] = id(i, jm, k); q[3] = id(i, jm, km); }
    else if (comp == 1) { q[0] = id(i, j, k); q[1] = id(im, j, k); q[2] = id(i, j, km); q[3] = id(im, j, km); }
    else { q[0] = id(i, j, k); q[1] = id(i, jm, k); q[2] = id(im, j, k); q[3] = id(im, jm, k); }
    for (int t = 0; t < 4; ++t) {
        e[t] = f.eps[q[t]];
        s[t] = f.sig[q[t]];
        l[t] = f.ell[q[t]];
    }
}

// Coefficients of one edge (as in the forward E pass): a, b and j = dt ell/mu0.
template <typename T>
__device__ __forceinline__ EdgeCoef<T> adj_coef(const T e4[4], const T s4[4], const T l4[4], T dt, T theta, T hdt)
{
    T eps, sig, ell;
    edge_material(e4, s4, l4, eps, sig, ell);
    const T sdt = sig * dt;
    const T inv = T(1) / (eps + theta * sdt);
    return {(eps - (T(1) - theta) * sdt) * inv, dt * inv, hdt * ell};
}

// Edge-local part of F2^T for component q of the edge at plane offset b, lane
// byte offsets ow (arrays of T) and od (FP64 gradient arrays), from values
// loaded by the caller: lJ and gL (superconducting edges only), gS, E^n, E'_pre.
template <typename T>
__device__ __forceinline__ void adj_edge_local(const AdjArgs<T> &A, int q, long long b, uint32_t ow, uint32_t od,
                                               const int pos[3], T lEq, const EdgeCoef<T> &k, T En, T Ep, T lJ,
                                               double gL, double gS)
{
    const int nx = A.f.g.nx, ny = A.f.g.ny;
    const T theta = A.f.theta, hdt = A.f.hdt;
    // PEC wall: E' = 0 there, so its adjoint does not propagate
    bool wall = false;
    for (int a = 0; a < 3; ++a)
        if (a != q && A.f.pml[a].on && pos[a] == 0) wall = true;
    const T lEp = wall ? T(0) : lEq;
    const T mu = k.cb * lEp;
    T ljt = T(0);
    if (k.cj > T(0)) {
        ljt = lJ - mu;
        stp(A.lJ[q] + b, ow, ljt);
        stp(A.gL[q] + b, od, gL + (double)hdt * (double)ljt * (double)En);
    }
    stp(A.gS[q] + b, od, gS - (double)lEp * (double)k.cb * ((double)theta * (double)Ep + (1.0 - (double)theta) * (double)En));
    stp(A.mu[q] + b, ow, mu);
    stp(A.lE[q] + b, ow, k.ca * lEp + k.cj * ljt);
    // E-side PML adjoint variables: tot = bn * stored + sg mu
    for (int a = 0; a < 3; ++a) {
        if (a == q) continue;
        const PmlAxis<T> &P = A.f.pml[a];
        if (!P.on) continue;
        const int sl = slab_slot(pos[a], P.lo, P.hi, P.n);
        if (sl < 0) continue;
        T *ps = A.lpsiE[a][psi_slot(q, a)];
        const long long pi = psi_index(P, a, nx, ny, pos[0], pos[1], pos[2], sl);
        ps[pi] = P.bn[pos[a]] * ps[pi] + T(curl_sign(q, a)) * mu;
    }
}

// z-marching like the forward E pass: the maps of plane k-1 and the z terms of
// the curl^T at k-1 are carried in registers, and the edge coefficients of a
// plane are formed one iteration ahead so that all loads of an iteration
// (including lJ and gL on superconducting edges) are issued before the first wait.
template <typename T, int TY, int TZ, bool CLS>
__global__ __launch_bounds__(kTileX *TY) void adj_edge_kernel(const AdjArgs<T> A)
{
    const int nx = A.f.g.nx, ny = A.f.g.ny, nz = A.f.g.nz;
    int i, j, k0, k1;
    if (!tile_of<TY, TZ>(nx, ny, nz, i, j, k0, k1)) return;
    const long long sxy = A.f.g.sxy;
    const int im = (i == 0) ? nx - 1 : i - 1;
    const int jm = (j == 0) ? ny - 1 : j - 1;
    // byte offsets inside one plane: each access is a plane base (scalar registers) plus a lane offset
    const uint32_t cell = uint32_t(j * nx + i);
    const uint32_t o00 = cell * sizeof(T), o10 = uint32_t(j * nx + im) * sizeof(T);
    const uint32_t o01 = uint32_t(jm * nx + i) * sizeof(T), o11 = uint32_t(jm * nx + im) * sizeof(T);
    const uint32_t od = cell * sizeof(double);
    const T rdx = A.f.rd[0], rdy = A.f.rd[1], rdz = A.f.rd[2];
    const T dt = A.f.dt, theta = A.f.theta, hdt = A.f.hdt;
    const bool theta_one = (theta == T(1));
    const int km0 = (k0 == 0) ? nz - 1 : k0 - 1;
    T whyz_m = T(0), whxz_m = T(0);
    if (A.doC) {
        const long long bm = (long long)km0 * sxy;
        whyz_m = w_face(A, 1, 2, i, j, km0, ldp(A.lH[1] + bm, o00));
        whxz_m = w_face(A, 0, 2, i, j, km0, ldp(A.lH[0] + bm, o00));
    }
    T pe00 = T(0), pe10 = T(0), pe01 = T(0), ps00 = T(0), ps10 = T(0), ps01 = T(0), pl00 = T(0), pl10 = T(0),
      pl01 = T(0);
    EdgeCoef<T> cq[3] = {};
    struct Maps {
        T e00, e10, e01, e11, s00, s10, s01, s11, l00, l10, l01, l11;
    };
    struct Classes {
        uint32_t x, y, z;
    };
    const uint32_t oc = cell * 2u;  // byte offset into a class plane
    auto load_maps = [&](int kk) {
        const long long b = opaque_offset((long long)kk * sxy);
        if constexpr (CLS) {
            return Classes{ldp(A.f.cls[0] + b, oc), ldp(A.f.cls[1] + b, oc), ldp(A.f.cls[2] + b, oc)};
        } else {
            const T *me = A.f.eps + b, *ms = A.f.sig + b, *ml = A.f.ell + b;
            return Maps{ldp(me, o00), ldp(me, o10), ldp(me, o01), ldp(me, o11),
                        ldp(ms, o00), ldp(ms, o10), ldp(ms, o01), ldp(ms, o11),
                        ldp(ml, o00), ldp(ml, o10), ldp(ml, o01), ldp(ml, o11)};
        }
    };
    auto coefs = [&](const auto &m) {
        if constexpr (CLS) {
            cq[0] = class_coef(A.f.ctab, m.x);
            cq[1] = class_coef(A.f.ctab, m.y);
            cq[2] = class_coef(A.f.ctab, m.z);
        } else {
            {   // Ex: cells (j,k), (j,k-1), (j-1,k), (j-1,k-1)
                const T e[4] = {m.e00, pe00, m.e01, pe01}, s[4] = {m.s00, ps00, m.s01, ps01},
                        l[4] = {m.l00, pl00, m.l01, pl01};
                cq[0] = adj_coef(e, s, l, dt, theta, hdt);
            }
            {   // Ey: cells (k,i), (k,i-1), (k-1,i), (k-1,i-1)
                const T e[4] = {m.e00, m.e10, pe00, pe10}, s[4] = {m.s00, m.s10, ps00, ps10},
                        l[4] = {m.l00, m.l10, pl00, pl10};
                cq[1] = adj_coef(e, s, l, dt, theta, hdt);
            }
            {   // Ez: cells (i,j), (i,j-1), (i-1,j), (i-1,j-1)
                const T e[4] = {m.e00, m.e01, m.e10, m.e11}, s[4] = {m.s00, m.s01, m.s10, m.s11},
                        l[4] = {m.l00, m.l01, m.l10, m.l11};
                cq[2] = adj_coef(e, s, l, dt, theta, hdt);
            }
            pe00 = m.e00; pe10 = m.e10; pe01 = m.e01;
            ps00 = m.s00; ps10 = m.s10; ps01 = m.s01;
            pl00 = m.l00; pl10 = m.l10; pl01 = m.l01;
        }
    };
    if (A.doA) {
        if constexpr (!CLS) {
            const Maps m = load_maps(km0);
            pe00 = m.e00; pe10 = m.e10; pe01 = m.e01;
            ps00 = m.s00; ps10 = m.s10; ps01 = m.s01;
            pl00 = m.l00; pl10 = m.l10; pl01 = m.l01;
        }
        coefs(load_maps(k0));
    }
    for (int k = k0; k < k1; ++k) {
        const long long b = opaque_offset((long long)k * sxy);
        T le[3] = {ldp(A.lE[0] + b, o00), ldp(A.lE[1] + b, o00), ldp(A.lE[2] + b, o00)};
        T hx0 = T(0), hy0 = T(0), hz0 = T(0), hz_ym = T(0), hz_xm = T(0), hx_ym = T(0), hy_xm = T(0);
        if (A.doC) {
            const T *Hx = A.lH[0] + b, *Hy = A.lH[1] + b, *Hz = A.lH[2] + b;
            hx0 = ldp(Hx, o00); hy0 = ldp(Hy, o00); hz0 = ldp(Hz, o00);
            hz_ym = ldp(Hz, o01); hz_xm = ldp(Hz, o10); hx_ym = ldp(Hx, o01); hy_xm = ldp(Hy, o10);
        }
        const EdgeCoef<T> kq[3] = {cq[0], cq[1], cq[2]};
        T En[3] = {}, Ep[3] = {}, lJ[3] = {};
        double gL[3] = {}, gS[3] = {};
        decltype(load_maps(0)) mn{};
        if (A.doA) {
            for (int q = 0; q < 3; ++q) {
                if (kq[q].cj > T(0)) {
                    lJ[q] = ldp(A.lJ[q] + b, o00);
                    gL[q] = ldp(A.gL[q] + b, od);
                }
            }
            for (int q = 0; q < 3; ++q) {
                // E^n enters the sigma gradient only through (1 - theta) E^n: with theta = 1 it is read
                // on superconducting edges only (the ell gradient)
                if (!theta_one || kq[q].cj > T(0)) En[q] = ldp(A.En[q] + b, o00);
                Ep[q] = ldp(A.Ep[q] + b, o00);
                gS[q] = ldp(A.gS[q] + b, od);
            }
            // E'_pre: the soft sources of this step taken out of the stored E^{m+1}
            for (int sidx = 0; sidx < A.nsrc; ++sidx) {
                if (k >= A.sbox[sidx][5] && k < A.sbox[sidx][6] && j >= A.sbox[sidx][3] && j < A.sbox[sidx][4] &&
                    i >= A.sbox[sidx][1] && i < A.sbox[sidx][2]) {
                    const int c = A.sbox[sidx][0];
                    const double g = A.sg[sidx];
                    // selects, not a store to Ep[c]: a variable index would move Ep to scratch memory
                    Ep[0] = (c == 0) ? (T)((double)Ep[0] - g) : Ep[0];
                    Ep[1] = (c == 1) ? (T)((double)Ep[1] - g) : Ep[1];
                    Ep[2] = (c == 2) ? (T)((double)Ep[2] - g) : Ep[2];
                }
            }
            // maps of the next plane (the last iteration re-reads its own plane and discards them)
            mn = load_maps(k + 1 < nz ? k + 1 : k);
        }
        if (A.doC) {
            const T whyz = w_face(A, 1, 2, i, j, k, hy0), whxz = w_face(A, 0, 2, i, j, k, hx0);
            // Ex: terms (Hy, z) and (Hz, y); Ey: (Hx, z) and (Hz, x); Ez: (Hx, y) and (Hy, x)
            le[0] += (whyz_m - whyz) * rdz + (w_face(A, 2, 1, i, jm, k, hz_ym) - w_face(A, 2, 1, i, j, k, hz0)) * rdy;
            le[1] += (whxz_m - whxz) * rdz + (w_face(A, 2, 0, im, j, k, hz_xm) - w_face(A, 2, 0, i, j, k, hz0)) * rdx;
            le[2] += (w_face(A, 0, 1, i, jm, k, hx_ym) - w_face(A, 0, 1, i, j, k, hx0)) * rdy +
                     (w_face(A, 1, 0, im, j, k, hy_xm) - w_face(A, 1, 0, i, j, k, hy0)) * rdx;
            whyz_m = whyz;
            whxz_m = whxz;
        }
        if (A.obj && i >= A.ob[0] && i < A.ob[1] && j >= A.ob[2] && j < A.ob[3] && k >= A.ob[4] && k < A.ob[5])
            le[A.ocomp] += (T)A.og;
        if (!A.doA) {
            for (int q = 0; q < 3; ++q) stp(A.lE[q] + b, o00, le[q]);
            continue;
        }
        const int pos[3] = {i, j, k};
        for (int q = 0; q < 3; ++q)
            adj_edge_local(A, q, b, o00, od, pos, le[q], kq[q], En[q], Ep[q], lJ[q], gL[q], gS[q]);
        coefs(mn);
    }
}

template <typename T>
__global__ void adj_initial_kick_kernel(const AdjArgs<T> A)
{
    const int nx = A.f.g.nx, ny = A.f.g.ny;
    const long long N = A.f.g.sxy * A.f.g.nz;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx);
        const long long r = c / nx;
        const int j = (int)(r % ny);
        const int k = (int)(r / ny);
        for (int q = 0; q < 3; ++q) {
            T e4[4], s4[4], l4[4];
            edge_cells(A.f, q, i, j, k, e4, s4, l4);
            T eps, sig, ell;
            edge_material(e4, s4, l4, eps, sig, ell);
            if (ell > T(0))
                A.gL[q][c] += -0.5 * (double)A.f.hdt * (double)A.lJ[q][c] * (double)A.En[q][c];
        }
    }
}

// Cell (i,j,k) owns 12 edges: Ex at (i, j+u, k+v), Ey at (i+u, j, k+v), Ez at
// (i+u, j+v, k).  The derivative of the edge rule gives weight 1/|S| to each
// superconducting cell of a superconducting edge (S its superconducting cells)
// and 1/4 to every cell of a normal edge (sigma only).
template <typename T>
__global__ void adj_edge_to_cell_kernel(const AdjArgs<T> A, double *gl_cell, double *gs_cell)
{
    const int nx = A.f.g.nx, ny = A.f.g.ny, nz = A.f.g.nz;
    const long long N = A.f.g.sxy * nz;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx);
        const long long r = c / nx;
        const int j = (int)(r % ny);
        const int k = (int)(r / ny);
        const bool self_sc = A.f.ell[c] > T(0);
        double gl = 0.0, gs = 0.0;
        for (int q = 0; q < 3; ++q)
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 2; ++v) {
                    int ei = i, ej = j, ek = k;
                    if (q == 0) { ej += u; ek += v; }
                    else if (q == 1) { ei += u; ek += v; }
                    else { ei += u; ej += v; }
                    if (ei == nx) ei = 0;
                    if (ej == ny) ej = 0;
                    if (ek == nz) ek = 0;
                    T e4[4], s4[4], l4[4];
                    edge_cells(A.f, q, ei, ej, ek, e4, s4, l4);
                    int nsc = 0;
                    for (int t = 0; t < 4; ++t) nsc += (l4[t] > T(0)) ? 1 : 0;
                    const long long e = ((long long)ek * ny + ej) * nx + ei;
                    if (nsc > 0) {
                        if (self_sc) {
                            gl += A.gL[q][e] / (double)nsc;
                            gs += A.gS[q][e] / (double)nsc;
                        }
                    } else {
                        gs += 0.25 * A.gS[q][e];
                    }
                }
        gl_cell[c] = gl;
        gs_cell[c] = gs;
    }
}

}  // namespace

// Both adjoint sweeps: 4 rows per block, the z run chosen as in the forward
// sweeps for at least 8192 wavefronts per launch.
constexpr int kAdjTileY = 4;
constexpr long long kAdjWaves = 8192;

template <typename T, int TY, int TZ>
static void launch_adj_tz(bool faces, const AdjArgs<T> &a, hipStream_t s)
{
    const dim3 blk(kTileX, TY), grd(tile_blocks(a.f.g, TY, TZ));
    if (faces)
        hipLaunchKernelGGL((adj_face_kernel<T, TY, TZ>), grd, blk, 0, s, a);
    else if (a.f.cls[0])
        hipLaunchKernelGGL((adj_edge_kernel<T, TY, TZ, true>), grd, blk, 0, s, a);
    else
        hipLaunchKernelGGL((adj_edge_kernel<T, TY, TZ, false>), grd, blk, 0, s, a);
}

template <typename T>
static hipError_t launch_adj_sweep(bool faces, const AdjArgs<T> &a, hipStream_t s)
{
    switch (pick_tile_z(a.f.g, kAdjTileY, kAdjWaves, 32)) {
    case 32: launch_adj_tz<T, kAdjTileY, 32>(faces, a, s); break;
    case 16: launch_adj_tz<T, kAdjTileY, 16>(faces, a, s); break;
    default: launch_adj_tz<T, kAdjTileY, 8>(faces, a, s); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_faces(const AdjArgs<T> &a, hipStream_t s)
{
    return launch_adj_sweep<T>(true, a, s);
}

template <typename T>
hipError_t launch_adj_edges(const AdjArgs<T> &a, hipStream_t s)
{
    return launch_adj_sweep<T>(false, a, s);
}

static int grid_blocks(long long N)
{
    const long long nb = (N + 255) / 256;
    return (int)(nb < 65536 ? nb : 65536);
}

template <typename T>
hipError_t launch_adj_initial_kick(const AdjArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL(adj_initial_kick_kernel<T>, dim3(grid_blocks(a.f.g.sxy * a.f.g.nz)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_edge_to_cell(const AdjArgs<T> &a, double *grad_ell, double *grad_sig, hipStream_t s)
{
    hipLaunchKernelGGL(adj_edge_to_cell_kernel<T>, dim3(grid_blocks(a.f.g.sxy * a.f.g.nz)), dim3(256), 0, s, a,
                       grad_ell, grad_sig);
    return hipGetLastError();
}

#define TFL_ADJ_INSTANTIATE(T)                                                        \
    template hipError_t launch_adj_faces<T>(const AdjArgs<T> &, hipStream_t);         \
    template hipError_t launch_adj_edges<T>(const AdjArgs<T> &, hipStream_t);         \
    template hipError_t launch_adj_initial_kick<T>(const AdjArgs<T> &, hipStream_t);  \
    template hipError_t launch_adj_edge_to_cell<T>(const AdjArgs<T> &, double *, double *, hipStream_t);

TFL_ADJ_INSTANTIATE(double)
TFL_ADJ_INSTANTIATE(float)

}  // namespace tfl

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
//               preceding step (mu = b lE, lJ, the ell gradient,
//               lE <- a lE + j lJ); mu is kept per step for a window of
//               steps, whose sigma gradient one more sweep then adds.
// Gradients with respect to the per-edge j = dt ell/mu0 and sigma follow from
// dJs'/d ell = dt E/mu0 and dE'/d sigma = -b (theta E'_pre + (1-theta) E).
// The multiplication of a PML adjoint variable by its decay b is applied when
// the variable is next read, so each sweep writes its variables once.
#include "fdtd_common.h"

namespace tfl {
namespace {

// Conventions written out in both sweeps: a curl term of component c
// differentiated along axis a enters with +1 when a = c+1 (mod 3) and -1 when
// a = c+2 (mod 3); the two CPML variables of axis a hold components a+1 and a+2
// (mod 3) in that order (x: y, z; y: z, x; z: x, y), indexed ((k ny + j) P + s)
// in x slabs, ((k P + s) nx + i) in y slabs and ((s ny + j) nx + i) in z slabs,
// with s the slot of the cell in the axis's pair of slabs.

// ---------------------------------------------------------------------------
// Face sweep: lH'' = lH + curl W (F2^T), then the H-side PML variables (F1^T)
// ---------------------------------------------------------------------------
// W of an E-side term inside a CPML slab (the adjoint of the stretched backward
// difference): sg kn mu + cn tot, with tot the stored E-side adjoint variable.
template <typename T>
__device__ __forceinline__ T w_slab(T sg, T kn, T cn, T muv, T tot)
{
    return sg * kn * muv + cn * tot;
}

// Outside the slabs W = sg mu.  Each axis has two terms per face position (the
// two edge components it differentiates), which share the slab test, the
// stretching coefficients and the index of their adjoint variables; the slab
// tests are hoisted (x per lane, y per row, z per plane), so the interior runs
// the stencil alone and the register count stays close to the H pass.
template <typename T, int TY, int TZ>
__global__ __launch_bounds__(kTileX *TY) void adj_face_kernel(const AdjArgs<T> A)
{
    const int nx = A.f.g.nx, ny = A.f.g.ny, nz = A.f.g.nz;
    int i, j, k0, k1;
    if (!tile_of<TY, TZ>(nx, ny, nz, i, j, k0, k1, zmix_of(A.f.pml[2], nz))) return;
    const long long sxy = A.f.g.sxy;
    const int ip = (i + 1 == nx) ? 0 : i + 1;
    const int jp = (j + 1 == ny) ? 0 : j + 1;
    const uint32_t o00 = uint32_t(j * nx + i) * sizeof(T), oxp = uint32_t(j * nx + ip) * sizeof(T);
    const uint32_t oyp = uint32_t(jp * nx + i) * sizeof(T);
    const uint32_t oi = uint32_t(i) * sizeof(T), oip = uint32_t(ip) * sizeof(T);
    const T rdx = A.f.rd[0], rdy = A.f.rd[1], rdz = A.f.rd[2], hdt = A.f.hdt;
    const T *mx = A.mu[0], *my = A.mu[1], *mz = A.mu[2];
    const PmlAxis<T> &px = A.f.pml[0], &py = A.f.pml[1], &pz = A.f.pml[2];
    // a wavefront is one row (blockDim.x = 64): j is uniform over it, so the y tests, the y
    // coefficients and the row parts of every adjoint-variable index are scalar
    const int jw = __builtin_amdgcn_readfirstlane(j), jpw = __builtin_amdgcn_readfirstlane(jp);
    // slab slots (-1 outside) of the lane's own and +1 positions along x, of the row and the next along y
    const int sxi = px.on ? slab_slot(i, px.lo, px.hi, nx) : -1;
    const int sxp = px.on ? slab_slot(ip, px.lo, px.hi, nx) : -1;
    const int syj = py.on ? slab_slot(jw, py.lo, py.hi, ny) : -1;
    const int syp = py.on ? slab_slot(jpw, py.lo, py.hi, ny) : -1;
    const uint32_t osxi = uint32_t(sxi) * sizeof(T), osxp = uint32_t(sxp) * sizeof(T);
    // the z terms W(Ey, z) and W(Ex, z) of plane k are those of plane k+1 one iteration earlier
    T wyz0, wxz0;
    {
        const long long b = (long long)k0 * sxy;
        const T my0 = ldo(my + b, o00), mx0 = ldo(mx + b, o00);
        wyz0 = my0;
        wxz0 = -mx0;
        const int sz = pz.on ? slab_slot(k0, pz.lo, pz.hi, nz) : -1;
        if (sz >= 0) {
            const long long r = ((long long)sz * ny + jw) * nx;
            const T kn = pz.kn[k0], cn = pz.cn[k0];
            wyz0 = w_slab(T(1), kn, cn, my0, ldo(A.lpsiE[2][1] + r, oi));
            wxz0 = w_slab(T(-1), kn, cn, mx0, ldo(A.lpsiE[2][0] + r, oi));
        }
    }
    for (int k = k0; k < k1; ++k) {
        const int kp = (k + 1 == nz) ? 0 : k + 1;
        const long long b = opaque_offset((long long)k * sxy), bp = opaque_offset((long long)kp * sxy);
        const T mx0 = ldo(mx + b, o00), my0 = ldo(my + b, o00), mz0 = ldo(mz + b, o00);
        const T my_kp = ldo(my + bp, o00), mx_kp = ldo(mx + bp, o00);
        const T mz_yp = ldo(mz + b, oyp), mz_xp = ldo(mz + b, oxp), mx_yp = ldo(mx + b, oyp), my_xp = ldo(my + b, oxp);
        const T lh0 = ldo(A.lH[0] + b, o00), lh1 = ldo(A.lH[1] + b, o00), lh2 = ldo(A.lH[2] + b, o00);
        // W outside the slabs: (Ey,z) +, (Ex,z) -, (Ez,y) -, (Ex,y) +, (Ez,x) +, (Ey,x) -
        T wyz1 = my_kp, wxz1 = -mx_kp;
        T wzy0 = -mz0, wzy1 = -mz_yp, wxy0 = mx0, wxy1 = mx_yp;
        T wzx0 = mz0, wzx1 = mz_xp, wyx0 = -my0, wyx1 = -my_xp;
        const int szk = pz.on ? slab_slot(k, pz.lo, pz.hi, nz) : -1;
        const int szp = pz.on ? slab_slot(kp, pz.lo, pz.hi, nz) : -1;
        // row bases of the adjoint variables: x slabs ((k ny + j) P + s), y slabs ((k P + s) nx + i)
        const long long rx = ((long long)k * ny + jw) * px.P;
        if (szp >= 0) {
            const long long r = ((long long)szp * ny + jw) * nx;
            const T kn = pz.kn[kp], cn = pz.cn[kp];
            wyz1 = w_slab(T(1), kn, cn, my_kp, ldo(A.lpsiE[2][1] + r, oi));
            wxz1 = w_slab(T(-1), kn, cn, mx_kp, ldo(A.lpsiE[2][0] + r, oi));
        }
        if (syj >= 0) {
            const long long r = ((long long)k * py.P + syj) * nx;
            const T kn = py.kn[jw], cn = py.cn[jw];
            wzy0 = w_slab(T(-1), kn, cn, mz0, ldo(A.lpsiE[1][0] + r, oi));
            wxy0 = w_slab(T(1), kn, cn, mx0, ldo(A.lpsiE[1][1] + r, oi));
        }
        if (syp >= 0) {
            const long long r = ((long long)k * py.P + syp) * nx;
            const T kn = py.kn[jpw], cn = py.cn[jpw];
            wzy1 = w_slab(T(-1), kn, cn, mz_yp, ldo(A.lpsiE[1][0] + r, oi));
            wxy1 = w_slab(T(1), kn, cn, mx_yp, ldo(A.lpsiE[1][1] + r, oi));
        }
        if (sxi >= 0) {
            const T kn = ldo(px.kn, oi), cn = ldo(px.cn, oi);
            wzx0 = w_slab(T(1), kn, cn, mz0, ldo(A.lpsiE[0][1] + rx, osxi));
            wyx0 = w_slab(T(-1), kn, cn, my0, ldo(A.lpsiE[0][0] + rx, osxi));
        }
        if (sxp >= 0) {
            const T kn = ldo(px.kn, oip), cn = ldo(px.cn, oip);
            wzx1 = w_slab(T(1), kn, cn, mz_xp, ldo(A.lpsiE[0][1] + rx, osxp));
            wyx1 = w_slab(T(-1), kn, cn, my_xp, ldo(A.lpsiE[0][0] + rx, osxp));
        }
        // lHx: terms (Ey, z) and (Ez, y); lHy: (Ex, z) and (Ez, x); lHz: (Ex, y) and (Ey, x)
        const T nh0 = lh0 + (wyz0 - wyz1) * rdz + (wzy0 - wzy1) * rdy;
        const T nh1 = lh1 + (wxz0 - wxz1) * rdz + (wzx0 - wzx1) * rdx;
        const T nh2 = lh2 + (wxy0 - wxy1) * rdy + (wyx0 - wyx1) * rdx;
        sto(A.lH[0] + b, o00, nh0);
        sto(A.lH[1] + b, o00, nh1);
        sto(A.lH[2] + b, o00, nh2);
        wyz0 = wyz1;
        wxz0 = wxz1;
        // H-side PML adjoint variables: tot = bh * stored + (-dt/mu0) sg lH'' for the two face
        // components each axis differentiates (x: Hy -, Hz +; y: Hz -, Hx +; z: Hx -, Hy +)
        if (sxi >= 0) {
            const T bh = ldo(px.bh, oi);
            T *p0 = A.lpsiH[0][0] + rx, *p1 = A.lpsiH[0][1] + rx;
            sto(p0, osxi, bh * ldo(p0, osxi) - hdt * T(-1) * nh1);
            sto(p1, osxi, bh * ldo(p1, osxi) - hdt * T(1) * nh2);
        }
        if (syj >= 0) {
            const long long r = ((long long)k * py.P + syj) * nx;
            const T bh = py.bh[jw];
            T *p0 = A.lpsiH[1][0] + r, *p1 = A.lpsiH[1][1] + r;
            sto(p0, oi, bh * ldo(p0, oi) - hdt * T(-1) * nh2);
            sto(p1, oi, bh * ldo(p1, oi) - hdt * T(1) * nh0);
        }
        if (szk >= 0) {
            const long long r = ((long long)szk * ny + jw) * nx;
            const T bh = pz.bh[k];
            T *p0 = A.lpsiH[2][0] + r, *p1 = A.lpsiH[2][1] + r;
            sto(p0, oi, bh * ldo(p0, oi) - hdt * T(-1) * nh0);
            sto(p1, oi, bh * ldo(p1, oi) - hdt * T(1) * nh1);
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

// Slab position of one edge row of the edge sweep: slots (-1 outside the slab)
// along x (per lane), y (per row) and z (per plane), and the row parts of the
// adjoint-variable indices (x slabs ((k ny + j) P + s), y slabs ((k P + s) nx + i),
// z slabs ((s ny + j) nx + i)), so each access is a scalar base plus a lane offset.
struct EdgeSlabs {
    int sx, sy, sz;
    uint32_t osx, oi;  // byte offsets of the x-slab slot and of column i (arrays of T)
    long long rx, ry, rz;
    int jw, k;
};

// Edge-local part of F2^T for component Q of the edge at plane offset b, lane
// byte offsets ow (arrays of T) and od (FP64 gradient arrays), from values
// loaded by the caller: lJ, gL and E^n (superconducting edges only).  The sigma
// gradient term of the edge, -mu (theta E'_pre + (1 - theta) E^n), is added by
// adj_grad_sigma_kernel from the stored mu of a window of steps.
// `wall`: the edge lies on the PEC wall of a CPML axis other than Q (E' = 0
// there, so its adjoint does not propagate).
template <int Q, typename T>
__device__ __forceinline__ void adj_edge_local(const AdjArgs<T> &A, long long b, uint32_t ow, uint32_t od, bool wall,
                                               const EdgeSlabs &sl, T lEq, const EdgeCoef<T> &k, T En, T lJ, double gL)
{
    const T hdt = A.f.hdt;
    const T lEp = wall ? T(0) : lEq;
    const T mu = k.cb * lEp;
    T ljt = T(0);
    if (k.cj > T(0)) {
        ljt = lJ - mu;
        sto(A.lJ[Q] + b, ow, ljt);
        sto(A.gL[Q] + b, od, gL + (double)hdt * (double)ljt * (double)En);
    }
    sto(A.mu[Q] + b, ow, mu);
    sto(A.lE[Q] + b, ow, k.ca * lEp + k.cj * ljt);
    // E-side PML adjoint variables of the two axes component Q is differentiated along:
    // tot = bn * stored + sg mu (x: Ey -, Ez +; y: Ez -, Ex +; z: Ex -, Ey +)
    if constexpr (Q != 0) {
        if (sl.sx >= 0) {
            T *ps = A.lpsiE[0][Q == 1 ? 0 : 1] + sl.rx;
            sto(ps, sl.osx, ldo(A.f.pml[0].bn, sl.oi) * ldo(ps, sl.osx) + T(Q == 1 ? -1 : 1) * mu);
        }
    }
    if constexpr (Q != 1) {
        if (sl.sy >= 0) {
            T *ps = A.lpsiE[1][Q == 0 ? 1 : 0] + sl.ry;
            sto(ps, sl.oi, A.f.pml[1].bn[sl.jw] * ldo(ps, sl.oi) + T(Q == 0 ? 1 : -1) * mu);
        }
    }
    if constexpr (Q != 2) {
        if (sl.sz >= 0) {
            T *ps = A.lpsiE[2][Q == 0 ? 0 : 1] + sl.rz;
            sto(ps, sl.oi, A.f.pml[2].bn[sl.k] * ldo(ps, sl.oi) + T(Q == 0 ? -1 : 1) * mu);
        }
    }
}

// WH of an H-side term inside a CPML slab (the adjoint of the stretched forward
// difference): -dt/mu0 sg kh lH + ch tot; outside the slabs -dt/mu0 sg lH.
template <typename T>
__device__ __forceinline__ T wh_slab(T sg, T hdt, T kh, T ch, T lh, T tot)
{
    return -hdt * sg * kh * lh + ch * tot;
}

// z-marching like the forward E pass: the maps of plane k-1 and the z terms of
// the curl^T at k-1 are carried in registers, and the edge coefficients of a
// plane are formed one iteration ahead so that all loads of an iteration
// (including lJ and gL on superconducting edges) are issued before the first wait.
// Slab tests are hoisted as in the face sweep (x per lane, y per row, z per plane).
template <typename T, int TY, int TZ, bool CLS>
__global__ __launch_bounds__(kTileX *TY) void adj_edge_kernel(const AdjArgs<T> A)
{
    const int nx = A.f.g.nx, ny = A.f.g.ny, nz = A.f.g.nz;
    int i, j, k0, k1;
    if (!tile_of<TY, TZ>(nx, ny, nz, i, j, k0, k1, zmix_of(A.f.pml[2], nz))) return;
    const long long sxy = A.f.g.sxy;
    const int im = (i == 0) ? nx - 1 : i - 1;
    const int jm = (j == 0) ? ny - 1 : j - 1;
    // byte offsets inside one plane: each access is a plane base (scalar registers) plus a lane offset
    const uint32_t cell = uint32_t(j * nx + i);
    const uint32_t o00 = cell * sizeof(T), o10 = uint32_t(j * nx + im) * sizeof(T);
    const uint32_t o01 = uint32_t(jm * nx + i) * sizeof(T), o11 = uint32_t(jm * nx + im) * sizeof(T);
    const uint32_t od = cell * sizeof(double);
    const uint32_t oi = uint32_t(i) * sizeof(T), oim = uint32_t(im) * sizeof(T);
    const T rdx = A.f.rd[0], rdy = A.f.rd[1], rdz = A.f.rd[2];
    const T dt = A.f.dt, theta = A.f.theta, hdt = A.f.hdt;
    const PmlAxis<T> &px = A.f.pml[0], &py = A.f.pml[1], &pz = A.f.pml[2];
    // a wavefront is one row (blockDim.x = 64): j is uniform over it
    const int jw = __builtin_amdgcn_readfirstlane(j), jmw = __builtin_amdgcn_readfirstlane(jm);
    const int sxi = px.on ? slab_slot(i, px.lo, px.hi, nx) : -1;
    const int sxm = px.on ? slab_slot(im, px.lo, px.hi, nx) : -1;
    const int syj = py.on ? slab_slot(jw, py.lo, py.hi, ny) : -1;
    const int sym = py.on ? slab_slot(jmw, py.lo, py.hi, ny) : -1;
    const uint32_t osxi = uint32_t(sxi) * sizeof(T), osxm = uint32_t(sxm) * sizeof(T);
    // PEC walls: node plane 0 of a CPML axis
    const bool wx = px.on && i == 0, wy = py.on && jw == 0;
    const int km0 = (k0 == 0) ? nz - 1 : k0 - 1;
    T whyz_m = T(0), whxz_m = T(0);
    if (A.doC) {
        const long long bm = (long long)km0 * sxy;
        const T hy = ldo(A.lH[1] + bm, o00), hx = ldo(A.lH[0] + bm, o00);
        whyz_m = -hdt * T(1) * hy;
        whxz_m = -hdt * T(-1) * hx;
        const int sz = pz.on ? slab_slot(km0, pz.lo, pz.hi, nz) : -1;
        if (sz >= 0) {
            const long long r = ((long long)sz * ny + jw) * nx;
            const T kh = pz.kh[km0], ch = pz.ch[km0];
            whyz_m = wh_slab(T(1), hdt, kh, ch, hy, ldo(A.lpsiH[2][1] + r, oi));
            whxz_m = wh_slab(T(-1), hdt, kh, ch, hx, ldo(A.lpsiH[2][0] + r, oi));
        }
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
            return Classes{ldo(A.f.cls[0] + b, oc), ldo(A.f.cls[1] + b, oc), ldo(A.f.cls[2] + b, oc)};
        } else {
            const T *me = A.f.eps + b, *ms = A.f.sig + b, *ml = A.f.ell + b;
            return Maps{ldo(me, o00), ldo(me, o10), ldo(me, o01), ldo(me, o11),
                        ldo(ms, o00), ldo(ms, o10), ldo(ms, o01), ldo(ms, o11),
                        ldo(ml, o00), ldo(ml, o10), ldo(ml, o01), ldo(ml, o11)};
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
        T le[3] = {ldo(A.lE[0] + b, o00), ldo(A.lE[1] + b, o00), ldo(A.lE[2] + b, o00)};
        T hx0 = T(0), hy0 = T(0), hz0 = T(0), hz_ym = T(0), hz_xm = T(0), hx_ym = T(0), hy_xm = T(0);
        if (A.doC) {
            const T *Hx = A.lH[0] + b, *Hy = A.lH[1] + b, *Hz = A.lH[2] + b;
            hx0 = ldo(Hx, o00); hy0 = ldo(Hy, o00); hz0 = ldo(Hz, o00);
            hz_ym = ldo(Hz, o01); hz_xm = ldo(Hz, o10); hx_ym = ldo(Hx, o01); hy_xm = ldo(Hy, o10);
        }
        const EdgeCoef<T> kq[3] = {cq[0], cq[1], cq[2]};
        T En[3] = {}, lJ[3] = {};
        double gL[3] = {};
        decltype(load_maps(0)) mn{};
        if (A.doA) {
            for (int q = 0; q < 3; ++q) {
                if (kq[q].cj > T(0)) {  // the ell gradient's terms: superconducting edges only
                    lJ[q] = ldo(A.lJ[q] + b, o00);
                    gL[q] = ldo(A.gL[q] + b, od);
                    En[q] = ldo(A.En[q] + b, o00);
                }
            }
            // maps of the next plane (the last iteration re-reads its own plane and discards them)
            mn = load_maps(k + 1 < nz ? k + 1 : k);
        }
        const int szk = pz.on ? slab_slot(k, pz.lo, pz.hi, nz) : -1;
        const long long rx = ((long long)k * ny + jw) * px.P;
        if (A.doC) {
            // WH outside the slabs: (Hy,z) +, (Hx,z) -, (Hz,y) -, (Hx,y) +, (Hz,x) +, (Hy,x) -
            T whyz = -hdt * T(1) * hy0, whxz = -hdt * T(-1) * hx0;
            T wzy_m = -hdt * T(-1) * hz_ym, wzy_0 = -hdt * T(-1) * hz0;
            T wxy_m = -hdt * T(1) * hx_ym, wxy_0 = -hdt * T(1) * hx0;
            T wzx_m = -hdt * T(1) * hz_xm, wzx_0 = -hdt * T(1) * hz0;
            T wyx_m = -hdt * T(-1) * hy_xm, wyx_0 = -hdt * T(-1) * hy0;
            if (szk >= 0) {
                const long long r = ((long long)szk * ny + jw) * nx;
                const T kh = pz.kh[k], ch = pz.ch[k];
                whyz = wh_slab(T(1), hdt, kh, ch, hy0, ldo(A.lpsiH[2][1] + r, oi));
                whxz = wh_slab(T(-1), hdt, kh, ch, hx0, ldo(A.lpsiH[2][0] + r, oi));
            }
            if (sym >= 0) {
                const long long r = ((long long)k * py.P + sym) * nx;
                const T kh = py.kh[jmw], ch = py.ch[jmw];
                wzy_m = wh_slab(T(-1), hdt, kh, ch, hz_ym, ldo(A.lpsiH[1][0] + r, oi));
                wxy_m = wh_slab(T(1), hdt, kh, ch, hx_ym, ldo(A.lpsiH[1][1] + r, oi));
            }
            if (syj >= 0) {
                const long long r = ((long long)k * py.P + syj) * nx;
                const T kh = py.kh[jw], ch = py.ch[jw];
                wzy_0 = wh_slab(T(-1), hdt, kh, ch, hz0, ldo(A.lpsiH[1][0] + r, oi));
                wxy_0 = wh_slab(T(1), hdt, kh, ch, hx0, ldo(A.lpsiH[1][1] + r, oi));
            }
            if (sxm >= 0) {
                const T kh = ldo(px.kh, oim), ch = ldo(px.ch, oim);
                wzx_m = wh_slab(T(1), hdt, kh, ch, hz_xm, ldo(A.lpsiH[0][1] + rx, osxm));
                wyx_m = wh_slab(T(-1), hdt, kh, ch, hy_xm, ldo(A.lpsiH[0][0] + rx, osxm));
            }
            if (sxi >= 0) {
                const T kh = ldo(px.kh, oi), ch = ldo(px.ch, oi);
                wzx_0 = wh_slab(T(1), hdt, kh, ch, hz0, ldo(A.lpsiH[0][1] + rx, osxi));
                wyx_0 = wh_slab(T(-1), hdt, kh, ch, hy0, ldo(A.lpsiH[0][0] + rx, osxi));
            }
            // Ex: terms (Hy, z) and (Hz, y); Ey: (Hx, z) and (Hz, x); Ez: (Hx, y) and (Hy, x)
            le[0] += (whyz_m - whyz) * rdz + (wzy_m - wzy_0) * rdy;
            le[1] += (whxz_m - whxz) * rdz + (wzx_m - wzx_0) * rdx;
            le[2] += (wxy_m - wxy_0) * rdy + (wyx_m - wyx_0) * rdx;
            whyz_m = whyz;
            whxz_m = whxz;
        }
        if (A.obj && i >= A.ob[0] && i < A.ob[1] && jw >= A.ob[2] && jw < A.ob[3] && k >= A.ob[4] && k < A.ob[5])
            le[A.ocomp] += (T)A.og;
        if (!A.doA) {
            for (int q = 0; q < 3; ++q) sto(A.lE[q] + b, o00, le[q]);
            continue;
        }
        const bool wz = pz.on && k == 0;
        const EdgeSlabs sl{sxi, syj, szk, osxi, oi, rx, ((long long)k * py.P + syj) * nx,
                           ((long long)szk * ny + jw) * nx, jw, k};
        adj_edge_local<0>(A, b, o00, od, wy || wz, sl, le[0], kq[0], En[0], lJ[0], gL[0]);
        adj_edge_local<1>(A, b, o00, od, wx || wz, sl, le[1], kq[1], En[1], lJ[1], gL[1]);
        adj_edge_local<2>(A, b, o00, od, wx || wy, sl, le[2], kq[2], En[2], lJ[2], gL[2]);
        coefs(mn);
    }
}

// The sigma gradient of a window of reverse steps, for each edge and in the order the edge sweeps
// ran those steps: gS -= mu (theta E'_pre + (1 - theta) E^n) in FP64, mu the step's b lE' stored by
// its edge sweep and E'_pre its E^{m+1} with the step's soft sources taken out (as the forward added
// them).  One sweep over a window replaces a read-modify-write of the FP64 accumulators per step.
template <typename T>
__global__ void adj_grad_sigma_kernel(const GradSigmaArgs<T> G)
{
    const long long N = G.g.sxy * G.g.nz;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        int i = 0, j = 0, k = 0;
        if (G.nsrc > 0) {
            i = (int)(c % G.g.nx);
            const long long r = c / G.g.nx;
            j = (int)(r % G.g.ny);
            k = (int)(r / G.g.ny);
        }
        for (int q = 0; q < 3; ++q) {
            double g = G.gS[q][c];
            for (int w = 0; w < G.nwin; ++w) {
                const T mu = G.mu[w][q][c];
                T Ep = G.Ep[w][q][c];
                for (int p = 0; p < G.nsrc; ++p) {
                    const int *b = G.sbox[p];
                    if (b[0] == q && k >= b[5] && k < b[6] && j >= b[3] && j < b[4] && i >= b[1] && i < b[2])
                        Ep = (T)((double)Ep - G.sg[w][p]);
                }
                const T En = G.En[w][q] ? G.En[w][q][c] : T(0);
                g = g - (double)mu * ((double)G.theta * (double)Ep + (1.0 - (double)G.theta) * (double)En);
            }
            G.gS[q][c] = g;
        }
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
hipError_t launch_adj_grad_sigma(const GradSigmaArgs<T> &g, hipStream_t s)
{
    if (g.nwin <= 0) return hipSuccess;
    hipLaunchKernelGGL(adj_grad_sigma_kernel<T>, dim3(grid_blocks(g.g.sxy * g.g.nz)), dim3(256), 0, s, g);
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
    template hipError_t launch_adj_grad_sigma<T>(const GradSigmaArgs<T> &, hipStream_t); \
    template hipError_t launch_adj_edge_to_cell<T>(const AdjArgs<T> &, double *, double *, hipStream_t);

TFL_ADJ_INSTANTIATE(double)
TFL_ADJ_INSTANTIATE(float)

}  // namespace tfl

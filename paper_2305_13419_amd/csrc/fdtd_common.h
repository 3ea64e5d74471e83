// Device helpers shared by the forward and adjoint sweeps.
#pragma once

#include "tfl_internal.h"

namespace tfl {

// Blocks are dealt to the 8 XCDs round robin; renumber them so that each XCD
// receives a contiguous range of tiles (neighbouring tiles share an L2).
static __device__ __forceinline__ int logical_block(int b, int nblocks)
{
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = b & 7, m = b >> 3;
    return x * q + min(x, r) + m;
}

static __device__ __forceinline__ int slab_slot(int i, int lo, int hi, int n)
{
    if (i < lo) return i;
    if (i >= n - hi) return lo + i - (n - hi);
    return -1;
}

template <typename T>
static __device__ __forceinline__ T inv_count(int c)
{
    return c == 1 ? T(1) : (c == 2 ? T(0.5) : (c == 3 ? T(1) / T(3) : T(0.25)));
}

// Per-edge material of the four cells q0..q3 sharing an edge (Sec. 3): if any
// cell is superconducting (ell > 0) the edge takes the mean over those cells,
// otherwise the mean over all four.  Summed in q order.
template <typename T>
static __device__ __forceinline__ void edge_material(const T e[4], const T s[4], const T l[4], T &eps, T &sig, T &ell)
{
    const bool anysc = (l[0] > T(0)) | (l[1] > T(0)) | (l[2] > T(0)) | (l[3] > T(0));
    T se = T(0), ss = T(0), sl = T(0);
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool use = !anysc || (l[q] > T(0));
        se += use ? e[q] : T(0);
        ss += use ? s[q] : T(0);
        sl += use ? l[q] : T(0);
        cnt += use ? 1 : 0;
    }
    const T ic = inv_count<T>(cnt);
    eps = T(kEps0) * (se * ic);
    sig = ss * ic;
    ell = sl * ic;
}

// Stretched derivative: d <- kappa^-1 d + psi, psi <- b psi + c d.
template <typename T>
static __device__ __forceinline__ T stretch(T d, T *psi, long long pidx, T b, T c, T kinv)
{
    const T p = b * psi[pidx] + c * d;
    psi[pidx] = p;
    return kinv * d + p;
}

template <typename T>
static __device__ __forceinline__ T stretch_virtual(T d, const T *psi, long long pidx, T b, T c, T kinv)
{
    const T p = b * psi[pidx] + c * d;
    return kinv * d + p;
}


}  // namespace tfl

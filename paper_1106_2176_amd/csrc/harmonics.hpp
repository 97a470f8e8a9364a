// harmonics.hpp -- device helpers shared by the uniform and adaptive L2P:
// the derivative vectors of a local expansion and its evaluation at a point.
#pragma once
#include "common.hpp"

namespace fmm {

// phi_hat = ell . rho(u),  E_hat = -(Gx, Gy, Gz) . rho(u)  (box units),
// where G are the coefficient vectors of the partial derivatives, from
//   d/dz R_n^m = R_{n-1}^m,  d/dx R_n^m = (R_{n-1}^{m+1} - R_{n-1}^{m-1})/2,
//   d/dy R_n^m = i (R_{n-1}^{m+1} + R_{n-1}^{m-1})/2.
template <typename T>
__device__ inline void getL(const T *ell, int P, int n, int m, T &re, T &im) {
    // complex L_n^m of an ell-type vector (m may be negative)
    re = T(0);
    im = T(0);
    if (n < 0 || n >= P) return;
    const int am = m < 0 ? -m : m;
    if (am > n) return;
    if (am == 0) {
        re = ell[n * n];
        return;
    }
    re = ell[n * n + 2 * am - 1] * T(0.5);
    im = -ell[n * n + 2 * am] * T(0.5);
    if (m < 0) {  // L^{-m} = (-1)^m conj(L^m)
        const T sg = (am & 1) ? T(-1) : T(1);
        re *= sg;
        im = -im * sg;
    }
}

// (ell, Gx, Gy, Gz) of slot c of an ell-type vector of order P
template <typename T, typename V>
__device__ inline V l2p_coef(const T *ell, int P, int c) {
    // slot c -> (j, v, part)
    int j = 0;
    while ((j + 1) * (j + 1) <= c) ++j;
    const int o = c - j * j;  // 0 .. 2j
    const int v = (o + 1) >> 1;
    const bool sine = o > 0 && (o & 1) == 0;
    V w;
    w.x = ell[c];
    w.y = w.z = w.w = T(0);
    if (j + 1 < P) {
        T r1, i1, r2, i2;
        getL(ell, P, j + 1, v - 1, r1, i1);
        getL(ell, P, j + 1, v + 1, r2, i2);
        // Gx = (L^{v-1} - L^{v+1})/2, Gy = i (L^{v-1} + L^{v+1})/2, Gz = L^v
        const T gxr = (r1 - r2) * T(0.5), gxi = (i1 - i2) * T(0.5);
        const T gyr = -(i1 + i2) * T(0.5), gyi = (r1 + r2) * T(0.5);
        T gzr, gzi;
        getL(ell, P, j + 1, v, gzr, gzi);
        if (v == 0) {
            w.y = gxr;
            w.z = gyr;
            w.w = gzr;
        } else if (!sine) {
            w.y = T(2) * gxr;
            w.z = T(2) * gyr;
            w.w = T(2) * gzr;
        } else {
            w.y = T(-2) * gxi;
            w.z = T(-2) * gyi;
            w.w = T(-2) * gzi;
        }
    }
    return w;
}

// phi_hat and the gradient sums (gx, gy, gz) = G . rho(u) of the slot
// vectors coef at u = (x, y, z); the harmonic loops are fully unrolled, so
// that every recurrence coefficient is a compile-time constant
template <int P, typename T, typename V>
__device__ __forceinline__ void l2p_point(const V *coef, T x, T y, T z, T &phi, T &gx, T &gy, T &gz) {
    const T r2 = x * x + y * y + z * z;
    phi = gx = gy = gz = T(0);
    T dr = T(1), di = T(0);
#pragma unroll
    for (int m = 0; m < P; ++m) {
        if (m > 0) {
            const T inv = T(-1) / T(2 * m);
            const T nr = (dr * x + di * y) * inv;
            const T ni = (di * x - dr * y) * inv;
            dr = nr;
            di = ni;
        }
        T ar = dr, ai = di, br = T(0), bi = T(0);
#pragma unroll
        for (int n = m; n < P; ++n) {
            T cr = ar, ci = ai;
            if (n == m + 1) {
                cr = z * ar;
                ci = z * ai;
            } else if (n > m + 1) {
                const T inv = T(1) / T((n - m) * (n + m));
                cr = (T(2 * n - 1) * z * ar - r2 * br) * inv;
                ci = (T(2 * n - 1) * z * ai - r2 * bi) * inv;
            }
            if (n > m) {
                br = ar;
                bi = ai;
                ar = cr;
                ai = ci;
            }
            if (m == 0) {
                const V w = coef[n * n];
                phi += w.x * cr;
                gx += w.y * cr;
                gy += w.z * cr;
                gz += w.w * cr;
            } else {
                const V w1 = coef[n * n + 2 * m - 1], w2 = coef[n * n + 2 * m];
                phi += w1.x * cr + w2.x * ci;
                gx += w1.y * cr + w2.y * ci;
                gy += w1.z * cr + w2.z * ci;
                gz += w1.w * cr + w2.w * ci;
            }
        }
    }
}

}  // namespace fmm

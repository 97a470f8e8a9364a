// common.hpp -- shared definitions of the gfx950 FMM library (device and host).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fmm.h"

namespace fmm {

// ---------------------------------------------------------------- layout
// Real coefficient vectors of length p^2 per box.  Degree n occupies slots
// n^2 .. n^2+2n: slot n^2 holds the m = 0 term, slots n^2+2m-1 and n^2+2m the
// cosine-like (real) and sine-like (imaginary) parts of order m = 1..n.
__host__ __device__ constexpr int cidx(int n, int m) { return n * n + (m == 0 ? 0 : 2 * m - 1); }

// Coefficient stride of a box in device arrays: p^2 rounded up to 8, so that
// an 8-wide bf16 MFMA operand piece never straddles two boxes.
__host__ __device__ constexpr int coef_stride(int p) { return (p * p + 7) & ~7; }
// Largest coefficient stride (p = FMM_P_MAX).
constexpr int kMaxStride = (FMM_P_MAX * FMM_P_MAX + 7) & ~7;
// Rows of an M2L operator: p^2 rounded up to the 16-row MFMA tile.
__host__ __device__ constexpr int m2l_rows(int p) { return (p * p + 15) & ~15; }

// Number of M2L offsets o in {-3..3}^3 with |o|_inf >= 2, and the ones a
// target of child class k (bit 0 x, 1 y, 2 z) interacts with: per axis the
// components -2-k_a .. 3-k_a, minus the 27 near offsets: 6^3 - 27 = 189.
constexpr int kNumOffsets = 316;
constexpr int kOffsetsPerClass = 189;

__host__ __device__ inline int offset_id343(int ox, int oy, int oz) {
    return (ox + 3) + 7 * ((oy + 3) + 7 * (oz + 3));
}

// ---------------------------------------------------------------- Morton
// Key bit 3b is bit b of the x box coordinate, 3b+1 of y, 3b+2 of z.
__host__ __device__ inline uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ inline uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x3ffu;
    return v;
}
__host__ __device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// ------------------------------------------------------- solid harmonics
// Regular solid harmonics R_n^m, the coefficients of the generating function
//   sum_{n,m} R_n^m(x) s^n t^m = exp(s (z + (x+iy)/(2t) - t (x-iy)/2)),
// so that R_n^m(a+b) = sum R_k^l(a) R_{n-k}^{m-l}(b) and
// 1/|x-y| = sum_{n,m} R_n^m(y) I_n^m(x) with I_n^m the irregular harmonics
// below.  For m >= 0:
//   R_0^0 = 1,  R_m^m = -(x - iy)/(2m) R_{m-1}^{m-1},  R_{m+1}^m = z R_m^m,
//   (n-m)(n+m) R_n^m = (2n-1) z R_{n-1}^m - r^2 R_{n-2}^m,
// and R_n^{-m} = (-1)^m conj(R_n^m).
// Writes the real vector rho (slots as cidx) for degrees 0..P-1.
template <typename T>
__host__ __device__ inline void regular_rho(int P, T x, T y, T z, T *rho) {
    const T r2 = x * x + y * y + z * z;
    T dr = T(1), di = T(0);
    for (int m = 0; m < P; ++m) {
        if (m > 0) {
            const T inv = T(-1) / T(2 * m);
            const T nr = (dr * x + di * y) * inv;
            const T ni = (di * x - dr * y) * inv;
            dr = nr;
            di = ni;
        }
        T ar = dr, ai = di;       // R_{m}^m
        T br = T(0), bi = T(0);   // R_{m-1}^m (= 0)
        for (int n = m; n < P; ++n) {
            T cr, ci;
            if (n == m) {
                cr = ar;
                ci = ai;
            } else if (n == m + 1) {
                cr = z * ar;
                ci = z * ai;
            } else {
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
                rho[n * n] = cr;
            } else {
                rho[n * n + 2 * m - 1] = cr;
                rho[n * n + 2 * m] = ci;
            }
        }
    }
}

// -------------------------------------------- binary16 M2L encoding scale
// Per-level maxima of the binary16 M2L encoding: one 32-bit slot per level.
constexpr int kLevelSlots = FMM_MAX_LEVEL + 1;
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
// Exponent e of the power-of-two scale 2^e that puts a level's largest
// scaled multipole (float bits `mx_bits`, non-negative) just below 2^14, so
// that its binary16 parts and their products stay in range; 0 for an
// all-zero level.  The pack kernel multiplies by 2^e, the M2L kernel divides
// its results by it.
__host__ __device__ inline int level_scale_exp(uint32_t mx_bits) {
    const float mx = __builtin_bit_cast(float, mx_bits);
    if (!(mx > 0.0f)) return 0;
    int e = 0;
    (void)frexpf(mx, &e);  // mx < 2^e
    return 14 - e;
}

// ----------------------------------------------------- particle records
// Sorted particles are stored relative to their leaf centre in units of the
// leaf width, u in [-1/2, 1/2]^3, with the charge:
//   mixed form: int4 (x, y, z) as 32-bit fixed point in units of 2^-30 leaf
//               widths, w = the FP32 charge's bits.  A neighbour shift is an
//               exact integer add (|u + d| <= 3/2 < 2), a pair difference an
//               exact integer subtraction rounded once to FP32.
//   FP64 form:  double4 (x, y, z, q).
constexpr double kFixScale = 1073741824.0;                 // 2^30
constexpr float kFixInv = 9.313225746154785156e-10f;       // 2^-30

__device__ inline void unpack_rec(const int4 r, float &x, float &y, float &z, float &q) {
    x = (float)r.x * kFixInv;
    y = (float)r.y * kFixInv;
    z = (float)r.z * kFixInv;
    q = __int_as_float(r.w);
}
__device__ inline void unpack_rec(const double4 r, double &x, double &y, double &z, double &q) {
    x = r.x;
    y = r.y;
    z = r.z;
    q = r.w;
}

// atomicMax on a word that many blocks share.  Atomics on one word run one
// after another where memory performs them, so a block whose value does not
// exceed the word's current one (a coherent read; the word only grows, so a
// stale read only lets an atomic through) skips its atomic.
__device__ __forceinline__ void atomic_max_shared(unsigned int *p, unsigned int v) {
    if (v > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, v);
}

// The last step of an evaluation for sorted particle i (Sec. 2.1, S11):
// phi = (near + far) / w and E = (near + far) / w^2 in FP64 (near and far in
// leaf units), the optional force q E, stored at the particle's place in the
// caller's order and dtype.  Shared by the combine kernel and the P2P kernel
// that ends with it.
struct Combine {
    const uint32_t *perm;
    const double4 *farf;  // NULL: no far field
    double inv_w;
    const void *q;
    void *phi, *vec;
    int flags;            // FMM_VEC_*
    int dtype;            // FMM_F32 / FMM_F64 of q, phi and vec
};
template <typename To>
__device__ __forceinline__ void combine_one(const Combine &c, int64_t i, const double4 a) {
    double4 b = make_double4(0, 0, 0, 0);
    if (c.farf) b = c.farf[i];
    const uint32_t o = c.perm[i];
    ((To *)c.phi)[o] = (To)((a.x + b.x) * c.inv_w);
    if (c.flags != FMM_VEC_NONE) {
        const double s = c.inv_w * c.inv_w * (c.flags == FMM_VEC_FORCE ? (double)((const To *)c.q)[o] : 1.0);
        To *const v = (To *)c.vec;
        v[3 * (size_t)o] = (To)((a.y + b.y) * s);
        v[3 * (size_t)o + 1] = (To)((a.z + b.z) * s);
        v[3 * (size_t)o + 2] = (To)((a.w + b.w) * s);
    }
}

}  // namespace fmm

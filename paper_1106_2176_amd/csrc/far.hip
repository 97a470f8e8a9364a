// far.hip -- P2M, M2M, L2L, L2P (Fig. 1 and Fig. 3), the M2L operand
// packing, the charge gather and the far + near combine.
//
// Per-level coefficient arrays are dense row-major grids [(2^l)^3][S] with
// S = coef_stride(p): a uniform tree needs no hash tables.  Box (i,j,k) of
// level l is row i + 2^l (j + 2^l k).  Leaves are visited in Morton order
// (the sorted particle order) and mapped to their row.
#include "kernels.hpp"

namespace fmm {

// Regular harmonics of one point written with a stride (LDS transposition)
template <int P, typename T>
__device__ __forceinline__ void rho_strided(T x, T y, T z, T *out, int stride) {
    const T r2 = x * x + y * y + z * z;
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
                out[(n * n) * stride] = cr;
            } else {
                out[(n * n + 2 * m - 1) * stride] = cr;
                out[(n * n + 2 * m) * stride] = ci;
            }
        }
    }
}

template <typename T> struct V4T;
template <> struct V4T<float> { using type = float4; };
template <> struct V4T<double> { using type = double4; };

// ---------------------------------------------------------------- P2M
// mu(leaf) = scale * sum_j q_j rho(u_j).  One 64-lane block per leaf; rounds
// of RS particles write their harmonics into LDS [coef][particle], then lanes
// sum rows (fixed order, deterministic).
template <int P, typename T>
__global__ __launch_bounds__(64) void k_p2m(int L, const typename V4T<T>::type *__restrict__ src,
                                            const uint32_t *__restrict__ start, T *__restrict__ M,
                                            double scale) {
    constexpr int P2 = P * P;
    constexpr int S = coef_stride(P);
    constexpr int RSraw = 32768 / (P2 * (int)sizeof(T));
    constexpr int RS = RSraw >= 64 ? 64 : RSraw >= 32 ? 32 : RSraw >= 16 ? 16 : 8;
    constexpr int NA = (P2 + 63) / 64;
    __shared__ T buf[P2 * (RS + 1)];
    const int lane = threadIdx.x;
    const uint32_t leaf = blockIdx.x;
    const uint32_t s0 = start[leaf], cnt = start[leaf + 1] - s0;
    const int side = 1 << L;
    const size_t row = (size_t)compact3(leaf) +
                       (size_t)side * (compact3(leaf >> 1) + (size_t)side * compact3(leaf >> 2));
    T acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = T(0);
    for (uint32_t c0 = 0; c0 < cnt; c0 += RS) {
        const int nr = (int)min((uint32_t)RS, cnt - c0);
        __syncthreads();
        if (lane < nr) {
            const auto v = src[s0 + c0 + lane];
            rho_strided<P, T>(v.x, v.y, v.z, buf + lane, RS + 1);
            const T q = v.w;
#pragma unroll
            for (int c = 0; c < P2; ++c) buf[c * (RS + 1) + lane] *= q;
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const int c = lane + 64 * a;
            if (c < P2) {
                T s = T(0);
                for (int j = 0; j < nr; ++j) s += buf[c * (RS + 1) + j];
                acc[a] += s;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        const int c = lane + 64 * a;
        if (c < P2) M[row * S + c] = (T)(acc[a] * (T)scale);
    }
}

// ---------------------------------------------------------------- L2P
// phi_hat = ell . rho(u),  E_hat = -(Gx, Gy, Gz) . rho(u)  (leaf units),
// where G are the coefficient vectors of the partial derivatives, from
//   d/dz R_n^m = R_{n-1}^m,  d/dx R_n^m = (R_{n-1}^{m+1} - R_{n-1}^{m-1})/2,
//   d/dy R_n^m = i (R_{n-1}^{m+1} + R_{n-1}^{m-1})/2.
// The same kernel evaluates an adjoint multipole vector at its particles.
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

template <int P, typename T>
__global__ __launch_bounds__(64) void k_l2p(int L, const typename V4T<T>::type *__restrict__ src,
                                            const uint32_t *__restrict__ start,
                                            const T *__restrict__ Lc, double4 *__restrict__ out) {
    constexpr int P2 = P * P;
    constexpr int S = coef_stride(P);
    using V = typename V4T<T>::type;
    __shared__ T ell[P2];
    __shared__ V coef[P2];  // (ell, Gx, Gy, Gz) per slot
    const int lane = threadIdx.x;
    const uint32_t leaf = blockIdx.x;
    const uint32_t s0 = start[leaf], cnt = start[leaf + 1] - s0;
    if (cnt == 0) return;
    const int side = 1 << L;
    const size_t row = (size_t)compact3(leaf) +
                       (size_t)side * (compact3(leaf >> 1) + (size_t)side * compact3(leaf >> 2));
    for (int c = lane; c < P2; c += 64) ell[c] = Lc[row * S + c];
    __syncthreads();
    for (int c = lane; c < P2; c += 64) {
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
        coef[c] = w;
    }
    __syncthreads();
    for (uint32_t j0 = lane; j0 < cnt; j0 += 64) {
        const V pt = src[s0 + j0];
        const T x = pt.x, y = pt.y, z = pt.z;
        const T r2 = x * x + y * y + z * z;
        T phi = T(0), gx = T(0), gy = T(0), gz = T(0);
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
        out[s0 + j0] = make_double4((double)phi, -(double)gx, -(double)gy, -(double)gz);
    }
}

// ------------------------------------------------------- M2M / L2L transfers
// UP:   out[parent][o]  = sum_c sum_k tab[c][k][o] in[child c][k]
// DOWN: out[child c][o] += sum_k tab[c][k][o] in[parent][k]
// tab is [8][p^2][p^2] (input-major, so threads = output rows read
// contiguously).  Tile of NP consecutive parents per block.
constexpr int kNP = 16;

template <typename Tin, typename Tout, typename Tc>
__global__ __launch_bounds__(256) void k_up(int P, int lp, const Tin *__restrict__ in,
                                            Tout *__restrict__ out, const Tc *__restrict__ tab) {
    extern __shared__ unsigned char smem_raw[];
    Tc *sm = (Tc *)smem_raw;  // [kNP][P2]
    const int P2 = P * P, S = coef_stride(P);
    const int np = 1 << lp;  // parents per axis
    const int64_t npar = (int64_t)np * np * np;
    const int64_t p0 = (int64_t)blockIdx.x * kNP;
    const int o = threadIdx.x;
    Tc acc[kNP];
#pragma unroll
    for (int a = 0; a < kNP; ++a) acc[a] = Tc(0);
    for (int c = 0; c < 8; ++c) {
        __syncthreads();
        for (int e = threadIdx.x; e < kNP * P2; e += blockDim.x) {
            const int a = e / P2, k = e - a * P2;
            const int64_t pid = p0 + a;
            Tc v = Tc(0);
            if (pid < npar) {
                const int64_t pi = pid % np, pj = (pid / np) % np, pk = pid / ((int64_t)np * np);
                const int64_t nc = 2 * (int64_t)np;
                const int64_t ci = 2 * pi + (c & 1), cj = 2 * pj + ((c >> 1) & 1),
                              ck = 2 * pk + ((c >> 2) & 1);
                v = (Tc)in[(ci + nc * (cj + nc * ck)) * S + k];
            }
            sm[a * P2 + k] = v;
        }
        __syncthreads();
        if (o < P2) {
            const Tc *t = tab + (size_t)c * P2 * P2 + o;
            for (int k = 0; k < P2; ++k) {
                const Tc w = t[(size_t)k * P2];
#pragma unroll
                for (int a = 0; a < kNP; ++a) acc[a] += w * sm[a * P2 + k];
            }
        }
    }
    if (o < P2)
#pragma unroll
        for (int a = 0; a < kNP; ++a)
            if (p0 + a < npar) out[(p0 + a) * S + o] = (Tout)acc[a];
}

template <typename Tin, typename Tout, typename Tc>
__global__ __launch_bounds__(256) void k_down(int P, int lp, const Tin *__restrict__ in,
                                              Tout *__restrict__ out, const Tc *__restrict__ tab) {
    extern __shared__ unsigned char smem_raw[];
    Tc *sm = (Tc *)smem_raw;  // [kNP][P2]
    const int P2 = P * P, S = coef_stride(P);
    const int np = 1 << lp;
    const int64_t npar = (int64_t)np * np * np;
    const int64_t p0 = (int64_t)blockIdx.x * kNP;
    const int o = threadIdx.x;
    for (int e = threadIdx.x; e < kNP * P2; e += blockDim.x) {
        const int a = e / P2, k = e - a * P2;
        sm[e] = (p0 + a < npar) ? (Tc)in[(p0 + a) * S + k] : Tc(0);
    }
    __syncthreads();
    if (o >= P2) return;
    const int64_t nc = 2 * (int64_t)np;
    for (int c = 0; c < 8; ++c) {
        Tc acc[kNP];
#pragma unroll
        for (int a = 0; a < kNP; ++a) acc[a] = Tc(0);
        const Tc *t = tab + (size_t)c * P2 * P2 + o;
        for (int k = 0; k < P2; ++k) {
            const Tc w = t[(size_t)k * P2];
#pragma unroll
            for (int a = 0; a < kNP; ++a) acc[a] += w * sm[a * P2 + k];
        }
#pragma unroll
        for (int a = 0; a < kNP; ++a) {
            const int64_t pid = p0 + a;
            if (pid >= npar) continue;
            const int64_t pi = pid % np, pj = (pid / np) % np, pk = pid / ((int64_t)np * np);
            const int64_t ci = 2 * pi + (c & 1), cj = 2 * pj + ((c >> 1) & 1),
                          ck = 2 * pk + ((c >> 2) & 1);
            Tout *dst = out + (ci + nc * (cj + nc * ck)) * S + o;
            *dst = (Tout)((Tc)*dst + acc[a]);
        }
    }
}

// -------------------------------------------------------------- M2L operand
// Pack level-l multipoles into a zero-padded grid with a 3-box halo
// [(n+6)^3][S], split into bf16 parts (mixed) or copied in FP64.
__device__ inline uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

template <typename Tin>
__global__ void k_pack_bf16(int P, int l, int parts, const Tin *__restrict__ in,
                            uint16_t *__restrict__ out, size_t part_stride) {
    const int S = coef_stride(P), P2 = P * P;
    const int64_t n = 1 << l, g = n + 6;
    const int64_t total = g * g * g * S;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int c = (int)(e % S);
    const int64_t b = e / S;
    const int64_t x = b % g - 3, y = (b / g) % g - 3, z = b / (g * g) - 3;
    double v = 0.0;
    if (c < P2 && x >= 0 && y >= 0 && z >= 0 && x < n && y < n && z < n)
        v = (double)in[(x + n * (y + n * z)) * S + c];
    for (int k = 0; k < parts; ++k) {
        const uint16_t h = bf16_rne((float)v);
        out[k * part_stride + e] = h;
        v -= (double)bf16_to_f(h);
    }
}

__global__ void k_pack_f64(int P, int l, const double *__restrict__ in, double *__restrict__ out) {
    const int S = coef_stride(P), P2 = P * P;
    const int64_t n = 1 << l, g = n + 6;
    const int64_t total = g * g * g * S;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int c = (int)(e % S);
    const int64_t b = e / S;
    const int64_t x = b % g - 3, y = (b / g) % g - 3, z = b / (g * g) - 3;
    double v = 0.0;
    if (c < P2 && x >= 0 && y >= 0 && z >= 0 && x < n && y < n && z < n)
        v = in[(x + n * (y + n * z)) * S + c];
    out[e] = v;
}

// ------------------------------------------------------------ gather/combine
template <typename Tq, typename V>
__global__ void k_gather_q(int64_t n, const uint32_t *__restrict__ perm, const Tq *__restrict__ q,
                           V *__restrict__ xyzq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    xyzq[i].w = (decltype(xyzq[i].w))q[perm[i]];
}

// phi = (near + far) / w,  E = (near + far) / w^2 in FP64, scattered to the
// caller's order; optional force q E.
template <typename To>
__global__ void k_combine(int64_t n, const uint32_t *__restrict__ perm,
                          const double4 *__restrict__ nearf, const double4 *__restrict__ farf,
                          double inv_w, const To *__restrict__ q, To *__restrict__ phi,
                          To *__restrict__ vec, int flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 a = nearf[i];
    double4 b = make_double4(0, 0, 0, 0);
    if (farf) b = farf[i];
    const uint32_t o = perm[i];
    phi[o] = (To)((a.x + b.x) * inv_w);
    if (flags != FMM_VEC_NONE) {
        const double s = inv_w * inv_w * (flags == FMM_VEC_FORCE ? (double)q[o] : 1.0);
        vec[3 * (size_t)o] = (To)((a.y + b.y) * s);
        vec[3 * (size_t)o + 1] = (To)((a.z + b.z) * s);
        vec[3 * (size_t)o + 2] = (To)((a.w + b.w) * s);
    }
}

// Adjoint combine: grad_q = phi_w, grad_x = -(w E_q + q E_w) (E_q given in
// the caller's order and units).
template <typename To>
__global__ void k_combine_grad(int64_t n, const uint32_t *__restrict__ perm,
                               const double4 *__restrict__ nearf, const double4 *__restrict__ farf,
                               double inv_w, const To *__restrict__ q, const To *__restrict__ w,
                               const To *__restrict__ Eq, To *__restrict__ gq, To *__restrict__ gx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 a = nearf[i];
    double4 b = make_double4(0, 0, 0, 0);
    if (farf) b = farf[i];
    const uint32_t o = perm[i];
    if (gq) gq[o] = (To)((a.x + b.x) * inv_w);
    if (gx) {
        const double s = inv_w * inv_w, qo = (double)q[o], wo = (double)w[o];
        for (int ax = 0; ax < 3; ++ax) {
            const double ew = ((ax == 0 ? a.y + b.y : ax == 1 ? a.z + b.z : a.w + b.w)) * s;
            gx[3 * (size_t)o + ax] = (To)(-(wo * (double)Eq[3 * (size_t)o + ax] + qo * ew));
        }
    }
}

// ------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
static hipError_t p2m_dispatch(int P, int L, const void *src, const uint32_t *start, T *M,
                               double scale, hipStream_t st) {
    const unsigned g = 1u << (3 * L);
    using V = typename V4T<T>::type;
    switch (P) {
#define CASE(PP) \
    case PP: k_p2m<PP, T><<<g, 64, 0, st>>>(L, (const V *)src, start, M, scale); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_p2m(int P, int L, bool f64, const void *src, const uint32_t *start, void *M,
                      double scale, hipStream_t st) {
    return f64 ? p2m_dispatch<double>(P, L, src, start, (double *)M, scale, st)
               : p2m_dispatch<float>(P, L, src, start, (float *)M, scale, st);
}

template <typename T>
static hipError_t l2p_dispatch(int P, int L, const void *src, const uint32_t *start, const T *Lc,
                               double4 *out, hipStream_t st) {
    const unsigned g = 1u << (3 * L);
    using V = typename V4T<T>::type;
    switch (P) {
#define CASE(PP) \
    case PP: k_l2p<PP, T><<<g, 64, 0, st>>>(L, (const V *)src, start, Lc, out); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_l2p(int P, int L, bool f64, const void *src, const uint32_t *start,
                      const void *Lc, double4 *out, hipStream_t st) {
    return f64 ? l2p_dispatch<double>(P, L, src, start, (const double *)Lc, out, st)
               : l2p_dispatch<float>(P, L, src, start, (const float *)Lc, out, st);
}

// in/out precisions: 0 = f32, 1 = f64; compute in FP64 when either is FP64
hipError_t launch_transfer(bool up, int P, int lp, int in_f64, int out_f64, const void *in,
                           void *out, const void *tab32, const void *tab64, hipStream_t st) {
    const int64_t np = (int64_t)1 << (3 * lp);
    const unsigned grid = nblk(np, kNP);
    const int threads = P * P <= 64 ? 64 : P * P <= 128 ? 128 : 256;
    const bool c64 = in_f64 || out_f64;
    const size_t sh = (size_t)kNP * P * P * (c64 ? 8 : 4);
#define LAUNCH(TI, TO, TC, TAB)                                                                    \
    do {                                                                                           \
        if (up)                                                                                    \
            k_up<TI, TO, TC><<<grid, threads, sh, st>>>(P, lp, (const TI *)in, (TO *)out,           \
                                                        (const TC *)TAB);                         \
        else                                                                                       \
            k_down<TI, TO, TC><<<grid, threads, sh, st>>>(P, lp, (const TI *)in, (TO *)out,         \
                                                          (const TC *)TAB);                       \
    } while (0)
    if (!c64)
        LAUNCH(float, float, float, tab32);
    else if (in_f64 && out_f64)
        LAUNCH(double, double, double, tab64);
    else if (in_f64)
        LAUNCH(double, float, double, tab64);
    else
        LAUNCH(float, double, double, tab64);
#undef LAUNCH
    return hipGetLastError();
}

hipError_t launch_pack(int P, int l, bool in_f64, int parts, const void *in, void *out,
                       size_t part_stride, hipStream_t st) {
    const int64_t g = ((int64_t)1 << l) + 6;
    const int64_t total = g * g * g * coef_stride(P);
    if (parts == 0) {
        k_pack_f64<<<nblk(total, 256), 256, 0, st>>>(P, l, (const double *)in, (double *)out);
    } else if (in_f64) {
        k_pack_bf16<double><<<nblk(total, 256), 256, 0, st>>>(P, l, parts, (const double *)in,
                                                               (uint16_t *)out, part_stride);
    } else {
        k_pack_bf16<float><<<nblk(total, 256), 256, 0, st>>>(P, l, parts, (const float *)in,
                                                              (uint16_t *)out, part_stride);
    }
    return hipGetLastError();
}

hipError_t launch_gather_q(int64_t n, int dtype, bool f64, const uint32_t *perm, const void *q,
                           void *xyzq, hipStream_t st) {
    if (dtype == FMM_F64) {
        if (f64)
            k_gather_q<double, double4><<<nblk(n, 256), 256, 0, st>>>(n, perm, (const double *)q,
                                                                       (double4 *)xyzq);
        else
            k_gather_q<double, float4><<<nblk(n, 256), 256, 0, st>>>(n, perm, (const double *)q,
                                                                      (float4 *)xyzq);
    } else {
        if (f64)
            k_gather_q<float, double4><<<nblk(n, 256), 256, 0, st>>>(n, perm, (const float *)q,
                                                                      (double4 *)xyzq);
        else
            k_gather_q<float, float4><<<nblk(n, 256), 256, 0, st>>>(n, perm, (const float *)q,
                                                                     (float4 *)xyzq);
    }
    return hipGetLastError();
}

hipError_t launch_combine(int64_t n, int dtype, const uint32_t *perm, const double4 *nearf,
                          const double4 *farf, double inv_w, const void *q, void *phi, void *vec,
                          int flags, hipStream_t st) {
    if (dtype == FMM_F64)
        k_combine<double><<<nblk(n, 256), 256, 0, st>>>(n, perm, nearf, farf, inv_w,
                                                         (const double *)q, (double *)phi,
                                                         (double *)vec, flags);
    else
        k_combine<float><<<nblk(n, 256), 256, 0, st>>>(n, perm, nearf, farf, inv_w,
                                                        (const float *)q, (float *)phi,
                                                        (float *)vec, flags);
    return hipGetLastError();
}

hipError_t launch_combine_grad(int64_t n, int dtype, const uint32_t *perm, const double4 *nearf,
                               const double4 *farf, double inv_w, const void *q, const void *w,
                               const void *Eq, void *gq, void *gx, hipStream_t st) {
    if (dtype == FMM_F64)
        k_combine_grad<double><<<nblk(n, 256), 256, 0, st>>>(
            n, perm, nearf, farf, inv_w, (const double *)q, (const double *)w, (const double *)Eq,
            (double *)gq, (double *)gx);
    else
        k_combine_grad<float><<<nblk(n, 256), 256, 0, st>>>(
            n, perm, nearf, farf, inv_w, (const float *)q, (const float *)w, (const float *)Eq,
            (float *)gq, (float *)gx);
    return hipGetLastError();
}

}  // namespace fmm

// far.hip -- P2M, M2M, L2L, L2P (Fig. 1 and Fig. 3), the M2L operand
// packing, the charge gather and the far + near combine.
//
// Per-level coefficient arrays are dense row-major grids [(2^l)^3][S] with
// S = coef_stride(p): a uniform tree needs no hash tables.  Box (i,j,k) of
// level l is row i + 2^l (j + 2^l k).  Leaves are visited in Morton order
// (the sorted particle order) and mapped to their row.
#include <type_traits>

#include "harmonics.hpp"
#include "kernels.hpp"

namespace fmm {

// Regular harmonics of NPT points, each times its `seed`, summed over the
// points in order and written with a stride (LDS transposition).  The
// recurrences are linear in the degree-0 term, so starting them from `seed`
// instead of 1 scales every harmonic by it.  The NPT recurrences are
// independent chains, which the latency-bound recurrence needs.
template <int P, typename T, int NPT>
__device__ __forceinline__ void rho_strided(const T (&x)[NPT], const T (&y)[NPT], const T (&z)[NPT],
                                            const T (&seed)[NPT], T *out, int stride) {
    T r2[NPT], dr[NPT], di[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        r2[j] = x[j] * x[j] + y[j] * y[j] + z[j] * z[j];
        dr[j] = seed[j];
        di[j] = T(0);
    }
#pragma unroll
    for (int m = 0; m < P; ++m) {
        T ar[NPT], ai[NPT], br[NPT], bi[NPT];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            if (m > 0) {
                const T inv = T(-1) / T(2 * m);
                const T nr = (dr[j] * x[j] + di[j] * y[j]) * inv;
                const T ni = (di[j] * x[j] - dr[j] * y[j]) * inv;
                dr[j] = nr;
                di[j] = ni;
            }
            ar[j] = dr[j];
            ai[j] = di[j];
            br[j] = T(0);
            bi[j] = T(0);
        }
#pragma unroll
        for (int n = m; n < P; ++n) {
            T sr = T(0), si = T(0);
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                T cr = ar[j], ci = ai[j];
                if (n == m + 1) {
                    cr = z[j] * ar[j];
                    ci = z[j] * ai[j];
                } else if (n > m + 1) {
                    const T inv = T(1) / T((n - m) * (n + m));
                    cr = (T(2 * n - 1) * z[j] * ar[j] - r2[j] * br[j]) * inv;
                    ci = (T(2 * n - 1) * z[j] * ai[j] - r2[j] * bi[j]) * inv;
                }
                if (n > m) {
                    br[j] = ar[j];
                    bi[j] = ai[j];
                    ar[j] = cr;
                    ai[j] = ci;
                }
                sr += cr;
                si += ci;
            }
            if (m == 0) {
                out[(n * n) * stride] = sr;
            } else {
                out[(n * n + 2 * m - 1) * stride] = sr;
                out[(n * n + 2 * m) * stride] = si;
            }
        }
    }
}

// particle record type of each form (see common.hpp)
template <typename T> struct V4T;
template <> struct V4T<float> { using type = int4; };
template <> struct V4T<double> { using type = double4; };

// ---------------------------------------------------------------- P2M
// mu(leaf) = scale * sum_j q_j rho(u_j).  Two Morton-consecutive leaves per
// 64-lane block, 32 lanes each: rounds of RS rows per leaf, each row the
// sum of q rho over two particles of one lane (two independent recurrence
// chains), written into LDS [coef][row]; then the 64 lanes sum the rows of
// both leaves' coefficients (fixed order, deterministic).
// Rows per round: 32 while the two leaves' LDS buffers stay within 16 KB,
// else 16 (up to 40 KB), else 8.  At p = 10 that is 16 in both forms: the
// 32-row FP32 buffer (26 KB) held a CU to six blocks, and the kernel is
// bound by the latency of the harmonic recurrence (16 rows: 62 -> 51 us at
// N = 1e6).
template <int P, typename T>
constexpr int p2m_rows() {
    constexpr int P2 = P * P;
    return 2 * P2 * 33 * (int)sizeof(T) <= 16384 ? 32 : 2 * P2 * 17 * (int)sizeof(T) <= 40960 ? 16 : 8;
}

// With perm given, each particle's charge is first gathered from the
// caller's array (q, FP64 when q64) through perm and stored into its record
// (the charge gather folded into P2M, which reads every record anyway).
__device__ __forceinline__ void set_charge(int4 &r, float q) { r.w = __float_as_int(q); }
__device__ __forceinline__ void set_charge(double4 &r, double q) { r.w = q; }

template <int P, typename T>
__global__ __launch_bounds__(64) void k_p2m(int L, typename V4T<T>::type *__restrict__ src,
                                            const uint32_t *__restrict__ start, T *__restrict__ M,
                                            double scale, const uint32_t *__restrict__ perm,
                                            const void *__restrict__ qin, int q64,
                                            uint32_t *__restrict__ clear) {
    // clear the per-level maxima that the level-max kernel (after M2M)
    // accumulates into
    if (clear && blockIdx.x == 0 && threadIdx.x < kLevelSlots) clear[threadIdx.x] = 0u;
    constexpr int P2 = P * P;
    constexpr int S = coef_stride(P);
    constexpr int RS = p2m_rows<P, T>();
    constexpr int NPT = 2;                  // particles per lane and round (rows hold their sums)
    constexpr int NI = (2 * P2 + 63) / 64;  // (leaf, coefficient) items per lane
    __shared__ T buf[2][P2 * (RS + 1)];
    const int lane = threadIdx.x, half = lane >> 5, hl = lane & 31;
    const uint32_t nleaf = 1u << (3 * L), l0 = 2 * blockIdx.x;
    // both leaves' ranges, uniform over the block (the second is empty past the end)
    const uint32_t sa = start[l0], sb = start[min(l0 + 1, nleaf)], se = start[min(l0 + 2, nleaf)];
    const uint32_t ca = sb - sa, cb = se - sb;
    const uint32_t my0 = half ? sb : sa, myc = half ? cb : ca;
    const uint32_t rounds = (max(ca, cb) + NPT * RS - 1) / (NPT * RS);
    T acc[NI];
#pragma unroll
    for (int a = 0; a < NI; ++a) acc[a] = T(0);
    for (uint32_t r = 0; r < rounds; ++r) {
        const uint32_t c0 = r * NPT * RS;
        if (r > 0) __syncthreads();
        // row hl of the round: particles c0 + hl + j RS (a missing one has
        // charge 0 and adds nothing)
        if (hl < RS && c0 + hl < myc) {
            T x[NPT], y[NPT], z[NPT], q[NPT];
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                x[j] = y[j] = z[j] = q[j] = T(0);
                if (c0 + hl + j * RS < myc) {
                    const uint32_t d = my0 + c0 + hl + j * RS;
                    auto rec = src[d];
                    if (perm) {
                        const uint32_t o = perm[d];
                        const T qv = q64 ? (T)((const double *)qin)[o] : (T)((const float *)qin)[o];
                        set_charge(rec, qv);
                        src[d] = rec;
                    }
                    unpack_rec(rec, x[j], y[j], z[j], q[j]);
                }
            }
            rho_strided<P, T, NPT>(x, y, z, q, buf[half] + hl, RS + 1);
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NI; ++a) {
            const int item = lane + 64 * a;
            if (item < 2 * P2) {
                const int h = item >= P2, c = item - h * P2;
                const uint32_t ch = h ? cb : ca;
                const int nr = ch > c0 ? (int)min((uint32_t)RS, ch - c0) : 0;
                const T *row = buf[h] + c * (RS + 1);
                T sum = T(0);
                for (int j = 0; j < nr; ++j) sum += row[j];
                acc[a] += sum;
            }
        }
    }
    const int side = 1 << L;
#pragma unroll
    for (int a = 0; a < NI; ++a) {
        const int item = lane + 64 * a;
        const int h = item >= P2, c = item - h * P2;
        const uint32_t leaf = l0 + h;
        if (item < 2 * P2 && leaf < nleaf) {
            const size_t row = (size_t)compact3(leaf) +
                               (size_t)side * (compact3(leaf >> 1) + (size_t)side * compact3(leaf >> 2));
            M[row * S + c] = (T)(acc[a] * (T)scale);
        }
    }
}

// ---------------------------------------------------------------- L2P
// phi_hat = ell . rho(u),  E_hat = -(Gx, Gy, Gz) . rho(u)  (leaf units),
// where G are the coefficient vectors of the partial derivatives, from
//   d/dz R_n^m = R_{n-1}^m,  d/dx R_n^m = (R_{n-1}^{m+1} - R_{n-1}^{m-1})/2,
//   d/dy R_n^m = i (R_{n-1}^{m+1} + R_{n-1}^{m-1})/2.
// The same kernel evaluates an adjoint multipole vector at its particles.
// Two Morton-consecutive leaves per 64-lane block, 32 lanes each (a leaf
// holds a few tens of particles).  The harmonic loops are fully unrolled, so
// that every recurrence coefficient is a compile-time constant.
template <int P, typename T, int FUSE>
__global__ __launch_bounds__(64) void k_l2p(int L, const typename V4T<T>::type *__restrict__ src,
                                            const uint32_t *__restrict__ start,
                                            const T *__restrict__ Lc, double4 *__restrict__ out, const Combine c) {
    constexpr int P2 = P * P;
    constexpr int S = coef_stride(P);
    constexpr int HL = 32;  // lanes per leaf
    using V = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
    __shared__ T ells[2][P2];
    __shared__ V coefs[2][P2];  // (ell, Gx, Gy, Gz) per slot
    const int hl = threadIdx.x & (HL - 1), half = threadIdx.x / HL;
    const uint32_t leaf = 2 * blockIdx.x + half;
    const bool live = leaf < (1u << (3 * L));  // the second half is idle at level 0
    const uint32_t s0 = live ? start[leaf] : 0u, cnt = live ? start[leaf + 1] - s0 : 0u;
    T *const ell = ells[half];
    V *const coef = coefs[half];
    const int side = 1 << L;
    const size_t row = (size_t)compact3(leaf) +
                       (size_t)side * (compact3(leaf >> 1) + (size_t)side * compact3(leaf >> 2));
    for (int c = hl; c < P2; c += HL) ell[c] = live ? Lc[row * S + c] : T(0);
    __syncthreads();
    for (int c = hl; c < P2; c += HL) coef[c] = l2p_coef<T, V>(ell, P, c);
    __syncthreads();
    for (uint32_t j0 = hl; j0 < cnt; j0 += HL) {
        // keep the coefficient reads in the loop: hoisted, all p^2 of them
        // would be held in registers
        __asm__ volatile("" ::: "memory");
        T x, y, z, qq;
        unpack_rec(src[s0 + j0], x, y, z, qq);
        T phi, gx, gy, gz;
        l2p_point<P, T, V>(coef, x, y, z, phi, gx, gy, gz);
        out[s0 + j0] = make_double4((double)phi, -(double)gx, -(double)gy, -(double)gz);
    }
    // FUSE (1: FP32, 2: FP64 caller data): the combine of the lane's far
    // values, just written, with the near field (c.farf holds the near
    // partials here), in a loop of its own so that the harmonics loop keeps
    // its registers
    if constexpr (FUSE != 0)
        for (uint32_t j0 = hl; j0 < cnt; j0 += HL)
            combine_one<std::conditional_t<FUSE == 2, double, float>>(c, s0 + j0, out[s0 + j0]);
}

// ------------------------------------------------------- M2M / L2L transfers
// UP:   out[parent][o]  = sum_c sum_k tab[c][k][o] in[child c][k]
// DOWN: out[child c][o] += sum_k tab[c][k][o] in[parent][k]
// tab is [8][p^2][p^2] input-major, padded with 4 p^2 + 16 zeros so that the
// last row tile and K step read in bounds.  Both are small GEMMs (rows =
// output coefficients, columns = parents) on the FP64 matrix cores whatever
// the storage precision of the levels: tiles of 16 output rows x 16
// consecutive parents, K in steps of 4 (v_mfma_f64_16x16x4_f64; A lane l
// holds row l%16, K l/16; B lane l holds K l/16, column l%16; result lane l,
// item i holds row l/16 + 4i of column l%16).
// A block is 8 waves over 16 parents, wave c taking child octant c, and NT
// row tiles starting at row tile blockIdx.y * NT (NT = all of them, or one
// for coarse levels with few parents): each B value a wave loads feeds NT
// MFMAs.  Every load is unconditional, so that the loads of a K step and the
// next are in flight together.
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <int P>
__device__ __forceinline__ int64_t child_box(int64_t par, int64_t np, int c) {
    const int64_t nc = 2 * np;
    const int64_t pi = par % np, pj = (par / np) % np, pk = par / (np * np);
    return (2 * pi + (c & 1)) + nc * ((2 * pj + ((c >> 1) & 1)) + nc * (2 * pk + (c >> 2)));
}

// acc[i] += A(row tile rt0 + i) * B over K = p^2 in steps of 4.  The loads
// of step s are issued D steps before its MFMAs (the K loop is unrolled and
// a scheduling barrier after each step keeps the loads where they are).  ap
// points at this lane's A element of row tile rt0 and K step 0; bload(s)
// returns this lane's B value of step s (k = 4 s + q < S, in bounds), masked
// here for k >= p^2.
template <int P, int NT, typename TB, typename BLoad>
__device__ __forceinline__ void transfer_gemm(f64x4_t (&acc)[NT], const double *__restrict__ ap,
                                              int q, BLoad bload) {
    constexpr int P2 = P * P, NKS = (P2 + 3) / 4;
    // one row tile (coarse levels, a few hundred parents): the wave's work is
    // a latency chain, so up to 16 steps of loads are kept in flight
    constexpr int D = NT == 1 ? (NKS < 16 ? NKS : 16) : NT <= 8 ? 3 : 2;
    double av[D][NT];
    TB bv[D];
#pragma unroll
    for (int s = 0; s < NKS + D; ++s) {
        if (s >= D) {
            const int t = s - D, d = t % D;
            const bool use = P2 % 4 == 0 || 4 * t + q < P2;
            const double b = use ? (double)bv[d] : 0.0;
#pragma unroll
            for (int i = 0; i < NT; ++i)
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[d][i], b, acc[i], 0, 0, 0);
        }
        if (s < NKS) {
            const int d = s % D;
            const double *a = ap + (size_t)4 * s * P2;
#pragma unroll
            for (int i = 0; i < NT; ++i) av[d][i] = a[16 * i];
            bv[d] = bload(s);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// UP: wave c accumulates child c's contribution (K = p^2); the 8 partial
// tiles are summed through LDS in child order 0..7.
template <int P, int NT, typename Tin, typename Tout>
__global__ __launch_bounds__(512) void k_up(int lp, const Tin *__restrict__ in,
                                            Tout *__restrict__ out, const double *__restrict__ tab) {
    constexpr int P2 = P * P, S = coef_stride(P);
    __shared__ f64x4_t red[7][64];
    const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int rt0 = blockIdx.y * NT;
    const int64_t np = (int64_t)1 << lp, npar = np * np * np;
    const int64_t par = (int64_t)blockIdx.x * 16 + col;
    const bool valid = par < npar;
    const Tin *bp = in + child_box<P>(valid ? par : 0, np, c) * S + q;
    const double *ap = tab + ((size_t)c * P2 + q) * P2 + rt0 * 16 + col;
    f64x4_t acc[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = f64x4_t{0, 0, 0, 0};
    // k = 4 s + q < S (S is a multiple of 8 >= p^2); the stride padding of a
    // coefficient row is not initialised and is masked in transfer_gemm
    transfer_gemm<P, NT, Tin>(acc, ap, q, [&](int s) { return bp[4 * s]; });
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        if (c > 0) red[c - 1][lane] = acc[i];
        __syncthreads();
        if (c == 0 && valid) {
            f64x4_t sum = acc[i];
#pragma unroll
            for (int w = 0; w < 7; ++w) sum += red[w][lane];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = (rt0 + i) * 16 + q + 4 * j;
                if (o < P2) out[par * S + o] = (Tout)sum[j];
            }
        }
        __syncthreads();
    }
}

// DOWN: the 16 parents' coefficients are staged in LDS (one contiguous run);
// wave c writes child c's rows.
template <int P, int NT, typename Tin, typename Tout>
__global__ __launch_bounds__(512) void k_down(int lp, const Tin *__restrict__ in,
                                              Tout *__restrict__ out, const double *__restrict__ tab) {
    constexpr int P2 = P * P, S = coef_stride(P);
    constexpr int SP = S + 1;  // odd stride: the 16 columns of a B read hit distinct banks
    __shared__ double sB[16 * SP];
    const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int rt0 = blockIdx.y * NT;
    const int64_t np = (int64_t)1 << lp, npar = np * np * np;
    const int64_t par0 = (int64_t)blockIdx.x * 16;
    const int ncol = (int)min((int64_t)16, npar - par0);
    for (int e = threadIdx.x; e < 16 * S; e += 512) {
        const int j = e / S, k = e - j * S;
        double v = 0.0;
        if (j < ncol && k < P2) v = (double)in[(par0 + j) * S + k];
        sB[j * SP + k] = v;
    }
    __syncthreads();
    const double *ap = tab + ((size_t)c * P2 + q) * P2 + rt0 * 16 + col;
    f64x4_t acc[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = f64x4_t{0, 0, 0, 0};
    const double *bcol = sB + col * SP + q;
    transfer_gemm<P, NT, double>(acc, ap, q, [&](int s) { return bcol[4 * s]; });
    if (col >= ncol) return;
    Tout *dst = out + child_box<P>(par0 + col, np, c) * S;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = (rt0 + i) * 16 + q + 4 * j;
            if (o < P2) dst[o] = (Tout)((double)dst[o] + acc[i][j]);
        }
    }
}

// -------------------------------------------------------------- M2L operand
// Pack the multipoles of levels 2..L into zero-padded grids with a 3-box
// halo [(n+6)^3][S]: FP64 for the plain form, FP32 for the mixed form (the
// M2L kernel splits it into bf16 parts in registers).  One launch for all
// levels: block b packs padded row b (a row is g boxes x S coefficients,
// contiguous in both arrays) of the level whose rows it falls in, four
// consecutive elements per thread.
template <typename Tin, typename Tout>
__device__ __forceinline__ void pack_row(int P, int n, int y, int z, const Tin *__restrict__ in,
                                         Tout *__restrict__ orow) {
    const int S = coef_stride(P), P2 = P * P, S4 = S / 4, g = n + 6;
    const bool yz = y >= 0 && z >= 0 && y < n && z < n;
    for (int e4 = threadIdx.x; e4 < g * S4; e4 += blockDim.x) {
        const int bx = e4 / S4, c = 4 * (e4 - bx * S4), x = bx - 3;
        Tout v[4] = {Tout(0), Tout(0), Tout(0), Tout(0)};
        if (yz && x >= 0 && x < n) {
            const Tin *src = in + ((size_t)x + (size_t)n * ((size_t)y + (size_t)n * z)) * S + c;
            if (c + 4 <= P2) {
#pragma unroll
                for (int k = 0; k < 4; ++k) v[k] = (Tout)src[k];
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (c + k < P2) v[k] = (Tout)src[k];
            }
        }
        Tout *dst = orow + (size_t)bx * S + c;
#pragma unroll
        for (int k = 0; k < 4; ++k) dst[k] = v[k];
    }
}

// 8 consecutive coefficients (a 32-byte aligned FP32 piece or a 64-byte
// aligned FP64 one) as FP32, in 16-byte loads
__device__ __forceinline__ void load8(const float *p, float (&v)[8]) {
    const float4 a = ((const float4 *)p)[0], b = ((const float4 *)p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
__device__ __forceinline__ void load8(const double *p, float (&v)[8]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double2 d = ((const double2 *)p)[k];
        v[2 * k] = (float)d.x;
        v[2 * k + 1] = (float)d.y;
    }
}

// binary16 encoding: one thread per 8-coefficient piece of a padded box; the
// piece is scaled (x rho_inv[c] x 2^e, e from the level's maximum) and split
// into two binary16 parts, stored hi8 then lo8 (32 bytes, the bytes of the
// FP32 piece it replaces).  Padding coefficients (rinv = 0 there) and halo
// boxes are zero.
template <typename Tin>
__device__ __forceinline__ void pack_row_h(int P, int n, int y, int z, const Tin *__restrict__ in,
                                           uint4 *__restrict__ orow, const float *rinv, float scale) {
    const int S = coef_stride(P), S8 = S / 8, g = n + 6;
    const bool yz = y >= 0 && z >= 0 && y < n && z < n;
    for (int e8 = threadIdx.x; e8 < g * S8; e8 += blockDim.x) {
        const int bx = e8 / S8, c = 8 * (e8 - bx * S8), x = bx - 3;
        float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (yz && x >= 0 && x < n) {
            load8(in + ((size_t)x + (size_t)n * ((size_t)y + (size_t)n * z)) * S + c, v);
            // padding coefficients are never written: select, do not multiply
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = rinv[c + k] != 0.0f ? v[k] * (rinv[c + k] * scale) : 0.0f;
        }
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const f32x2_t a = {v[2 * k], v[2 * k + 1]};
            const f16x2_t h = __builtin_convertvector(a, f16x2_t);
            const f16x2_t lo = __builtin_convertvector(a - __builtin_convertvector(h, f32x2_t), f16x2_t);
            hw[k] = __builtin_bit_cast(uint32_t, h);
            lw[k] = __builtin_bit_cast(uint32_t, lo);
        }
        uint4 *dst = orow + 2 * ((size_t)bx * S8 + c / 8);
        dst[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        dst[1] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
}

template <typename Tout>
__global__ __launch_bounds__(256) void k_pack(int P, PackPlan pl) {
    const int64_t b = blockIdx.x;
    int li = 0;
#pragma unroll
    for (int j = 1; j < kMaxPackLev; ++j)
        if (j < pl.nlev && b >= pl.row0[j]) li = j;
    // uniform selection from the per-level arrays (no dynamic indexing of
    // the argument struct)
    int l = pl.level[0], in_f64 = pl.in_f64[0];
    int64_t r0 = pl.row0[0];
    const void *in = pl.in[0];
    void *out = pl.out[0];
#pragma unroll
    for (int j = 1; j < kMaxPackLev; ++j)
        if (j == li) {
            l = pl.level[j];
            in_f64 = pl.in_f64[j];
            r0 = pl.row0[j];
            in = pl.in[j];
            out = pl.out[j];
        }
    const int n = 1 << l, g = n + 6;
    const int row = (int)(b - r0);  // z g + y of the padded grid (< 2^31)
    const int y = row % g - 3, z = row / g - 3;
    Tout *orow = (Tout *)out + (size_t)row * g * coef_stride(P);
    if (pl.lmax) {  // binary16 parts (Tout = float: the same bytes per piece)
        __shared__ float rinv[kMaxStride];
        for (int c = threadIdx.x; c < coef_stride(P); c += blockDim.x) rinv[c] = pl.rho_inv[c];
        __syncthreads();
        const float scale = ldexpf(1.0f, level_scale_exp(pl.lmax[l]));
        if (in_f64)
            pack_row_h(P, n, y, z, (const double *)in, (uint4 *)orow, rinv, scale);
        else
            pack_row_h(P, n, y, z, (const float *)in, (uint4 *)orow, rinv, scale);
    } else if (in_f64)
        pack_row(P, n, y, z, (const double *)in, orow);
    else
        pack_row(P, n, y, z, (const float *)in, orow);
}

// Largest |M_c rho_inv[c]| over the boxes of each level 2..L (binary16
// encoding of the M2L operands), as an atomic maximum on the float's bits
// (non-negative floats order like their bit patterns) into lmax[level],
// which P2M cleared.  Block b covers kLevelMaxChunk consecutive elements of
// the level whose blocks it falls in, four (one 16-byte load, within one
// box) per thread and step; padding coefficients (c >= p^2, never written)
// are skipped.
constexpr int kLevelMaxChunk = 256 * 32;
__global__ __launch_bounds__(256) void k_level_max(int P, PackPlan pl) {
    const int64_t b = blockIdx.x;
    int li = 0;
#pragma unroll
    for (int j = 1; j < kMaxPackLev; ++j)
        if (j < pl.nlev && b >= pl.blk0[j]) li = j;
    int l = pl.level[0], in_f64 = pl.in_f64[0];
    int64_t b0 = pl.blk0[0];
    const void *in = pl.in[0];
#pragma unroll
    for (int j = 1; j < kMaxPackLev; ++j)
        if (j == li) {
            l = pl.level[j];
            in_f64 = pl.in_f64[j];
            b0 = pl.blk0[j];
            in = pl.in[j];
        }
    __shared__ float rinv[kMaxStride];
    const int S = coef_stride(P), P2 = P * P, S4 = S / 4;
    for (int c = threadIdx.x; c < S; c += 256) rinv[c] = c < P2 ? pl.rho_inv[c] : 0.0f;
    __syncthreads();
    const int64_t ng = ((int64_t)1 << (3 * l)) * S4;  // 4-element groups of the level
    const int64_t g0 = (b - b0) * (kLevelMaxChunk / 4), g1 = min(ng, g0 + kLevelMaxChunk / 4);
    int cg = (int)((g0 + threadIdx.x) % S4);  // group's position in its box
    const int step = 256 % S4;
    // eight steps of four elements per thread, every load issued before the
    // first use (the steps past the level's end read nothing and add zeros)
    constexpr int STEPS = kLevelMaxChunk / 4 / 256;
    float v[STEPS][4];
    // (a step past the end reads the chunk's first group, in bounds, and is
    // zeroed afterwards: no branch between the loads)
    if (in_f64) {
        double2 d[STEPS][2];
#pragma unroll
        for (int t = 0; t < STEPS; ++t) {
            const int64_t gi = g0 + threadIdx.x + 256 * t, gs = gi < g1 ? gi : g0;
            d[t][0] = ((const double2 *)in)[2 * gs];
            d[t][1] = ((const double2 *)in)[2 * gs + 1];
        }
#pragma unroll
        for (int t = 0; t < STEPS; ++t) {
            const bool in_range = g0 + threadIdx.x + 256 * t < g1;
            v[t][0] = in_range ? (float)d[t][0].x : 0.0f;
            v[t][1] = in_range ? (float)d[t][0].y : 0.0f;
            v[t][2] = in_range ? (float)d[t][1].x : 0.0f;
            v[t][3] = in_range ? (float)d[t][1].y : 0.0f;
        }
    } else {
        float4 f[STEPS];
#pragma unroll
        for (int t = 0; t < STEPS; ++t) {
            const int64_t gi = g0 + threadIdx.x + 256 * t;
            f[t] = ((const float4 *)in)[gi < g1 ? gi : g0];
        }
#pragma unroll
        for (int t = 0; t < STEPS; ++t) {
            const bool in_range = g0 + threadIdx.x + 256 * t < g1;
            v[t][0] = in_range ? f[t].x : 0.0f;
            v[t][1] = in_range ? f[t].y : 0.0f;
            v[t][2] = in_range ? f[t].z : 0.0f;
            v[t][3] = in_range ? f[t].w : 0.0f;
        }
    }
    float mx = 0.0f;
#pragma unroll
    for (int t = 0; t < STEPS; ++t) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (4 * cg + k < P2) mx = fmaxf(mx, fabsf(v[t][k]) * rinv[4 * cg + k]);
        cg += step;
        if (cg >= S4) cg -= S4;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    __shared__ float wmax[4];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
        atomic_max_shared(pl.lmax + l, __float_as_uint(mx));  // hundreds of blocks a level
    }
}

// ------------------------------------------------------------ gather/combine
template <typename Tq>
__global__ void k_gather_q64(int64_t n, const uint32_t *__restrict__ perm, const Tq *__restrict__ q,
                             double4 *__restrict__ xyzq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    xyzq[i].w = (double)q[perm[i]];
}
template <typename Tq>
__global__ void k_gather_q32(int64_t n, const uint32_t *__restrict__ perm, const Tq *__restrict__ q,
                             int4 *__restrict__ xyzq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    xyzq[i].w = __float_as_int((float)q[perm[i]]);
}

// phi = (near + far) / w,  E = (near + far) / w^2 in FP64, scattered to the
// caller's order; optional force q E.
template <typename To>
__global__ void k_combine(int64_t n, const double4 *__restrict__ nearf, const Combine c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    combine_one<To>(c, i, nearf[i]);
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
static hipError_t p2m_dispatch(int P, int L, void *src, const uint32_t *start, T *M,
                               double scale, const uint32_t *perm, const void *q, int q64,
                               uint32_t *clear, hipStream_t st) {
    const unsigned g = ((1u << (3 * L)) + 1) / 2;  // two leaves per block
    using V = typename V4T<T>::type;
    switch (P) {
#define CASE(PP) \
    case PP: k_p2m<PP, T><<<g, 64, 0, st>>>(L, (V *)src, start, M, scale, perm, q, q64, clear); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_p2m(int P, int L, bool f64, void *src, const uint32_t *start, void *M,
                      double scale, const uint32_t *perm, const void *q, int q_dtype,
                      uint32_t *clear, hipStream_t st) {
    const int q64 = q_dtype == FMM_F64;
    return f64 ? p2m_dispatch<double>(P, L, src, start, (double *)M, scale, perm, q, q64, clear, st)
               : p2m_dispatch<float>(P, L, src, start, (float *)M, scale, perm, q, q64, clear, st);
}

template <typename T>
static hipError_t l2p_dispatch(int P, int L, const void *src, const uint32_t *start, const T *Lc,
                               double4 *out, const Combine &c, hipStream_t st) {
    const unsigned g = ((1u << (3 * L)) + 1) / 2;  // two leaves per block
    using V = typename V4T<T>::type;
    switch (P) {
#define CASE(PP)                                                                            \
    case PP:                                                                                \
        if (!c.phi)                                                                         \
            k_l2p<PP, T, 0><<<g, 64, 0, st>>>(L, (const V *)src, start, Lc, out, c);        \
        else if (c.dtype == FMM_F64)                                                        \
            k_l2p<PP, T, 2><<<g, 64, 0, st>>>(L, (const V *)src, start, Lc, out, c);        \
        else                                                                                \
            k_l2p<PP, T, 1><<<g, 64, 0, st>>>(L, (const V *)src, start, Lc, out, c);        \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_l2p(int P, int L, bool f64, const void *src, const uint32_t *start,
                      const void *Lc, double4 *out, const Combine *fuse, hipStream_t st) {
    const Combine c = fuse ? *fuse : Combine{};
    return f64 ? l2p_dispatch<double>(P, L, src, start, (const double *)Lc, out, c, st)
               : l2p_dispatch<float>(P, L, src, start, (const float *)Lc, out, c, st);
}

// in/out storage precisions: 0 = f32, 1 = f64 (the arithmetic is FP64)
template <int P>
static void transfer_p(bool up, int lp, int in_f64, int out_f64, const void *in, void *out,
                       const double *tab, hipStream_t st) {
    const int64_t np = (int64_t)1 << (3 * lp);
    // blocks of 16 parents; all row tiles in one block when there are enough
    // parent tiles to fill the chip, else one row tile per block
    constexpr int NRT = (P * P + 15) / 16;
    const unsigned ncol = (unsigned)((np + 15) / 16);
    const bool all = ncol >= 128;
    const dim3 grid(ncol, all ? 1u : (unsigned)NRT);
#define LAUNCH(TI, TO)                                                                           \
    do {                                                                                         \
        if (up && all)                                                                           \
            k_up<P, NRT, TI, TO><<<grid, 512, 0, st>>>(lp, (const TI *)in, (TO *)out, tab);     \
        else if (up)                                                                             \
            k_up<P, 1, TI, TO><<<grid, 512, 0, st>>>(lp, (const TI *)in, (TO *)out, tab);       \
        else if (all)                                                                            \
            k_down<P, NRT, TI, TO><<<grid, 512, 0, st>>>(lp, (const TI *)in, (TO *)out, tab);   \
        else                                                                                     \
            k_down<P, 1, TI, TO><<<grid, 512, 0, st>>>(lp, (const TI *)in, (TO *)out, tab);     \
    } while (0)
    if (in_f64 && out_f64)
        LAUNCH(double, double);
    else if (in_f64)
        LAUNCH(double, float);
    else if (out_f64)
        LAUNCH(float, double);
    else
        LAUNCH(float, float);
#undef LAUNCH
}

hipError_t launch_transfer(bool up, int P, int lp, int in_f64, int out_f64, const void *in,
                           void *out, const void *tab32, const void *tab64, hipStream_t st) {
    (void)tab32;
    const double *tab = (const double *)tab64;
    switch (P) {
#define CASE(PP) \
    case PP: transfer_p<PP>(up, lp, in_f64, out_f64, in, out, tab, st); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// f64_out: FP64 grid (plain form); otherwise FP32 (mixed form)
hipError_t launch_pack(int P, bool f64_out, const PackPlan &pl_in, hipStream_t st) {
    if (pl_in.nlev < 1 || pl_in.nlev > kMaxPackLev) return hipErrorInvalidValue;
    if (pl_in.lmax && (f64_out || !pl_in.rho_inv)) return hipErrorInvalidValue;
    PackPlan pl = pl_in;
    if (pl.lmax) {
        // the binary16 scale of each level needs its maximum first
        int64_t nb = 0;
        for (int i = 0; i < pl.nlev; ++i) {
            pl.blk0[i] = nb;
            nb += ((((int64_t)1 << (3 * pl.level[i])) * coef_stride(P)) + kLevelMaxChunk - 1) / kLevelMaxChunk;
        }
        pl.blk0[pl.nlev] = nb;
        k_level_max<<<(unsigned)nb, 256, 0, st>>>(P, pl);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const unsigned rows = (unsigned)pl.row0[pl.nlev];
    if (f64_out)
        k_pack<double><<<rows, 256, 0, st>>>(P, pl);
    else
        k_pack<float><<<rows, 256, 0, st>>>(P, pl);
    return hipGetLastError();
}

hipError_t launch_gather_q(int64_t n, int dtype, bool f64, const uint32_t *perm, const void *q,
                           void *xyzq, hipStream_t st) {
    if (dtype == FMM_F64) {
        if (f64)
            k_gather_q64<double><<<nblk(n, 256), 256, 0, st>>>(n, perm, (const double *)q, (double4 *)xyzq);
        else
            k_gather_q32<double><<<nblk(n, 256), 256, 0, st>>>(n, perm, (const double *)q, (int4 *)xyzq);
    } else {
        if (f64)
            k_gather_q64<float><<<nblk(n, 256), 256, 0, st>>>(n, perm, (const float *)q, (double4 *)xyzq);
        else
            k_gather_q32<float><<<nblk(n, 256), 256, 0, st>>>(n, perm, (const float *)q, (int4 *)xyzq);
    }
    return hipGetLastError();
}

hipError_t launch_combine(int64_t n, const double4 *nearf, const Combine &c, hipStream_t st) {
    if (c.dtype == FMM_F64)
        k_combine<double><<<nblk(n, 256), 256, 0, st>>>(n, nearf, c);
    else
        k_combine<float><<<nblk(n, 256), 256, 0, st>>>(n, nearf, c);
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

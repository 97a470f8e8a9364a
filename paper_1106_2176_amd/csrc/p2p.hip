// p2p.hip -- near-field particle-to-particle kernel (the P2P of Sec. 3.1,
// the kernel the paper vectorises, Sec. 3.2).
//
// One 64-lane wavefront per target leaf.  The 27 (or fewer, at the domain
// boundary) near leaves are streamed through LDS in tiles of 64 sources,
// consecutive neighbour leaves packed into one tile, already shifted into
// the target leaf's frame: coordinates are stored in
// leaf units relative to the leaf centre, so a source in the neighbour at
// offset d is at u_j + d and every difference is formed from numbers of
// magnitude <= 3/2 (no cancellation against absolute positions).
// Lane mapping: a chunk of up to 128 targets is covered by G = ceil(nt/2)
// lanes holding two targets each, replicated into K = 64/G groups that take
// every K-th source of a tile (source split); group partials are summed at
// the end.  Each source read from LDS feeds two pair interactions.
// Mixed form: positions are 32-bit fixed point (units of 2^-30 leaf widths),
// so a pair difference is an exact integer subtraction rounded once to FP32;
// the pair arithmetic is FP32 with the hardware reciprocal square root in
// these raw units, per-tile FP32 partial sums are merged into FP64, and the
// sums are rescaled at the end (phi by 2^30, E by 2^60, both exact).
// Plain form: FP64 throughout; 1/sqrt from the hardware estimate refined by
// one Newton-Raphson step y <- y + y (1 - r^2 y^2) / 2 (near field against
// the FP64 oracle: rel-L2 5e-16 in phi, 1e-15 in E; a second step changes
// that to 4e-16 and 5e-16 and costs 15% of the kernel's time).
// Pairs in the target's own leaf are masked when r^2 == 0 (the particle
// itself and exact duplicates contribute nothing); pairs with other leaves
// add a tiny constant to r^2 (one raw unit^2 = 2^-60 leaf widths^2 in the
// mixed form, 1e-200 in FP64), which keeps a quantisation-induced r^2 == 0
// finite and changes no pair farther apart than 1e-6 leaf widths by more
// than 1e-6 relative.
#include <climits>
#include <type_traits>

#include "kernels.hpp"

namespace fmm {

template <bool SELF>
__device__ __forceinline__ void pair_fix(int xi, int yi, int zi, const int4 s, float &phi, float &ex,
                                         float &ey, float &ez) {
    const float dx = (float)(xi - s.x), dy = (float)(yi - s.y), dz = (float)(zi - s.z);
    float r2 = SELF ? dx * dx : __builtin_fmaf(dx, dx, 1.0f);
    r2 = __builtin_fmaf(dy, dy, r2);
    r2 = __builtin_fmaf(dz, dz, r2);
    float rinv = __builtin_amdgcn_rsqf(r2);
    if (SELF) rinv = r2 > 0.0f ? rinv : 0.0f;
    const float qr = __int_as_float(s.w) * rinv;
    phi += qr;
    const float qr3 = qr * (rinv * rinv);
    ex = __builtin_fmaf(qr3, dx, ex);
    ey = __builtin_fmaf(qr3, dy, ey);
    ez = __builtin_fmaf(qr3, dz, ez);
}

template <bool SELF>
__device__ __forceinline__ void pair_f64(double xi, double yi, double zi, const double4 s,
                                         double &phi, double &ex, double &ey, double &ez) {
    const double dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
    double r2 = SELF ? dx * dx : __builtin_fma(dx, dx, 1e-200);
    r2 = __builtin_fma(dy, dy, r2);
    r2 = __builtin_fma(dz, dz, r2);
    double y = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2 * y, y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    if (SELF) y = r2 > 0.0 ? y : 0.0;
    const double qr = s.w * y;
    phi += qr;
    const double qr3 = qr * (y * y);
    ex = __builtin_fma(qr3, dx, ex);
    ey = __builtin_fma(qr3, dy, ey);
    ez = __builtin_fma(qr3, dz, ez);
}

template <typename T> struct V4;
template <> struct V4<float> { using type = int4; };
template <> struct V4<double> { using type = double4; };

template <typename T> struct Acc;
template <> struct Acc<float> { using type = float; };
template <> struct Acc<double> { using type = double; };

template <bool SELF>
__device__ __forceinline__ void pair(const int4 t, const int4 s, float &phi, float &ex, float &ey,
                                     float &ez) {
    pair_fix<SELF>(t.x, t.y, t.z, s, phi, ex, ey, ez);
}
template <bool SELF>
__device__ __forceinline__ void pair(const double4 t, const double4 s, double &phi, double &ex,
                                     double &ey, double &ez) {
    pair_f64<SELF>(t.x, t.y, t.z, s, phi, ex, ey, ez);
}

// |u| <= 1/2 - 2^-30 after quantisation, so shifted sources lie within
// +-(3/2) 2^30 and every target - source difference within +-(2^31 - 1).
__device__ __forceinline__ int4 shifted(int4 v, int dx, int dy, int dz) {
    v.x += dx * (1 << 30);
    v.y += dy * (1 << 30);
    v.z += dz * (1 << 30);
    return v;
}
__device__ __forceinline__ double4 shifted(double4 v, int dx, int dy, int dz) {
    v.x += (double)dx;
    v.y += (double)dy;
    v.z += (double)dz;
    return v;
}

// Synchronisation of one wave's LDS traffic: a wave's LDS operations run in
// order, so a compiler fence suffices (no block barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Chunks of a target leaf.  A chunk of c targets uses G = ceil(c/2) lanes
// (two targets each) times K = 64/G source groups, so one tile of 64 sources
// costs about ceil(64/K) steps of the pair loop (37 instructions for its two
// pairs) plus ~45 for staging the tile and merging the partial sums.  When
// G K falls well short of 64 (34 targets: G = 17, K = 3, 51 lanes busy) a
// leaf costs less as two chunks that fill the lanes (32 + 2), although each
// walks the neighbours again.  The next chunk is the size that minimises the
// cost of it and one more chunk for the rest, among the remainder itself
// and the sizes that fill the lanes; this matches the best split into any
// number of chunks for leaves of up to ~100 targets.  The per-tile overhead
// of 200 is measured rather than counted: with 45 (the instructions alone),
// C2 split most leaves of 25-40 targets and its P2P slowed by 5%.
// Splitting is used only for trees of at least 8^7 leaves (split): there it
// took the C4 P2P from 58.9 to 55.1 ms, while at C2 (8^5 leaves, four waves
// per wave slot) the split leaves' longer waves set the kernel's tail and
// it ran 2% slower.
__device__ __forceinline__ int p2p_tile_cost(int c) {
    const int g = (c + 1) >> 1, k = max(1, 64 / g);
    return ((64 + k - 1) / k) * 37 + 200;
}
__device__ __forceinline__ int p2p_next_chunk(int n, bool split) {
    if (!split) return min(n, 128);
    constexpr int kFill[7] = {128, 64, 42, 32, 24, 20, 16};
    int best = n <= 128 ? n : 128, bestv = n <= 128 ? p2p_tile_cost(n) : INT_MAX;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const int c = kFill[i];
        if (c >= n || n - c > 128) continue;
        const int v = p2p_tile_cost(c) + p2p_tile_cost(n - c);
        if (v < bestv) {
            bestv = v;
            best = c;
        }
    }
    return best;
}

// src: sorted particles (u_x, u_y, u_z, q) in leaf units; start: Morton leaf
// ranges; out: (phi, E) per sorted particle in leaf units (phi * w, E * w^2),
// or with FUSE (1: FP32, 2: FP64 caller data) the combine of each target
// with its far field, stored in the caller's order (out unused).
// NP = 1: one wave per target leaf.  NP = 3 (few leaves, too few waves to
// hide the serial walk over 27 neighbours): a block of three waves per
// target leaf, wave w taking the neighbour plane dz = w - 1; wave 0 adds the
// three planes' sums in plane order.
// The one-wave FP32 kernel asks for eight waves per SIMD (64 registers; its
// LDS, 5 KB, allows as many): the loop is bound by instruction issue and LDS
// latency, which more resident waves hide.  The FP64 kernel holds twice the
// data per pair and fits four (128 registers).
template <typename T>
constexpr int p2p_waves(int NP) { return NP == 1 ? (sizeof(T) == 4 ? 8 : 4) : 1; }
template <typename T, int NP, int FUSE>
__global__ __launch_bounds__(64 * NP)
__attribute__((amdgpu_waves_per_eu(p2p_waves<T>(NP), NP == 1 ? p2p_waves<T>(NP) : 10))) void k_p2p(int L, uint32_t per_xcd,
                                                 const typename V4<T>::type *__restrict__ src,
                                                 const uint32_t *__restrict__ start,
                                                 double4 *__restrict__ out, const Combine c) {
    using V = typename V4<T>::type;
    __shared__ V tiles[NP][64];
    __shared__ double4 reds[NP][2][64];
    __shared__ double4 planes[NP > 1 ? (NP - 1) * 128 : 1];  // [plane - 1][a/b][target]
    const int lane = NP == 1 ? (int)threadIdx.x : (int)threadIdx.x & 63;
    const int wave = NP == 1 ? 0 : (int)threadIdx.x >> 6;
    V *const tile = tiles[wave];
    double4 (*const red)[64] = reds[wave];
    auto sync = [&]() __attribute__((always_inline)) {
        if constexpr (NP == 1)
            __syncthreads();
        else
            wave_sync();
    };
    // a target's sums in leaf units: stored, or combined with the far field
    auto emit = [&](uint32_t i, double4 v) __attribute__((always_inline)) {
        if constexpr (sizeof(T) == 4) {  // raw fixed-point units -> leaf units
            const double s1 = kFixScale, s3 = kFixScale * kFixScale;
            v = make_double4(v.x * s1, v.y * s3, v.z * s3, v.w * s3);
        }
        if constexpr (FUSE == 0)
            out[i] = v;
        else
            combine_one<std::conditional_t<FUSE == 2, double, float>>(c, i, v);
    };
    // blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
    // run of Morton leaves so its L2 holds the shared neighbour sources
    const uint32_t leaf = (blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
    const uint32_t nleaf = 1u << (3 * L);
    if (leaf >= nleaf) return;
    const uint32_t t0 = start[leaf], nt = start[leaf + 1] - t0;
    if (nt == 0) return;
    const int side = 1 << L;
    const int ix = (int)compact3(leaf), iy = (int)compact3(leaf >> 1), iz = (int)compact3(leaf >> 2);

    for (uint32_t tc = 0, step = 0; tc < nt; tc += step) {
        const int ntc = p2p_next_chunk((int)(nt - tc), L >= 7);
        step = (uint32_t)ntc;
        const int G = (ntc + 1) >> 1;
        const int K = 64 / G;
        const int grp = lane / G, r = lane - grp * G;
        const bool act = grp < K;
        const bool hasb = act && (r + G < ntc);
        const V ta = src[t0 + tc + min(r, ntc - 1)];
        const V tb = src[t0 + tc + (hasb ? r + G : min(r, ntc - 1))];
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0, b0 = 0, b1 = 0, b2 = 0, b3 = 0;
        // pairs with the tile's first nsc sources, FP32 partial sums merged
        // into FP64; every compute ends with a sync, so the tile is free for
        // the next write
        auto compute = [&](int nsc, auto selfc) __attribute__((always_inline)) {
            constexpr bool SELF = decltype(selfc)::value;
            T pa0 = 0, pa1 = 0, pa2 = 0, pa3 = 0, pb0 = 0, pb1 = 0, pb2 = 0, pb3 = 0;
            if (act) {
                for (int j = grp; j < nsc; j += K) {
                    const V sj = tile[j];
                    pair<SELF>(ta, sj, pa0, pa1, pa2, pa3);
                    pair<SELF>(tb, sj, pb0, pb1, pb2, pb3);
                }
            }
            a0 += (double)pa0;
            a1 += (double)pa1;
            a2 += (double)pa2;
            a3 += (double)pa3;
            b0 += (double)pb0;
            b1 += (double)pb1;
            b2 += (double)pb2;
            b3 += (double)pb3;
            sync();
        };
        // other leaves are packed back to back into the tile (each source
        // already shifted into the target's frame) and computed when the
        // next one would not fit; the target's own leaf, whose pairs need
        // the r^2 == 0 mask, takes tiles of its own
        int pend = 0;
        auto flush = [&]() __attribute__((always_inline)) {
            if (pend > 0) {
                sync();
                compute(pend, std::false_type{});
                pend = 0;
            }
        };
        for (int dz = -1; dz <= 1; ++dz) {
            if (NP > 1 && dz != wave - 1) continue;
            if (iz + dz < 0 || iz + dz >= side) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                if (iy + dy < 0 || iy + dy >= side) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    if (ix + dx < 0 || ix + dx >= side) continue;
                    const uint32_t s = morton3(ix + dx, iy + dy, iz + dz);
                    const uint32_t s0 = start[s], ns = start[s + 1] - s0;
                    if ((dx | dy | dz) == 0) {
                        flush();
                        for (uint32_t sc = 0; sc < ns; sc += 64) {
                            const int nsc = (int)min(64u, ns - sc);
                            if (lane < nsc) tile[lane] = src[s0 + sc + lane];
                            sync();
                            compute(nsc, std::true_type{});
                        }
                        continue;
                    }
                    for (uint32_t sc = 0; sc < ns; sc += 64) {
                        const int nsc = (int)min(64u, ns - sc);
                        if (pend + nsc > 64) flush();
                        if (lane < nsc) tile[pend + lane] = shifted(src[s0 + sc + lane], dx, dy, dz);
                        pend += nsc;
                    }
                }
            }
        }
        flush();
        // sum the K source-split groups (fixed order: group 0, 1, ..., K-1)
        sync();
        red[0][lane] = make_double4(a0, a1, a2, a3);
        red[1][lane] = make_double4(b0, b1, b2, b3);
        sync();
        if constexpr (NP == 1) {
            // the two targets one after the other (fewer live registers)
            if (grp == 0)
                for (int h = 0; h < (hasb ? 2 : 1); ++h) {
                    double4 sh = red[h][r];
                    for (int g = 1; g < K; ++g) {
                        const double4 x = red[h][g * G + r];
                        sh.x += x.x; sh.y += x.y; sh.z += x.z; sh.w += x.w;
                    }
                    emit(t0 + tc + r + h * G, sh);
                }
            continue;
        }
        double4 sa = make_double4(0, 0, 0, 0), sb = sa;
        if (grp == 0) {
            sa = red[0][r];
            sb = red[1][r];
            for (int g = 1; g < K; ++g) {
                const double4 xa = red[0][g * G + r], xb = red[1][g * G + r];
                sa.x += xa.x; sa.y += xa.y; sa.z += xa.z; sa.w += xa.w;
                sb.x += xb.x; sb.y += xb.y; sb.z += xb.z; sb.w += xb.w;
            }
        }
        {
            // every wave reaches both barriers (the chunk loop is the same
            // in all waves of the block)
            __syncthreads();
            if (wave > 0 && grp == 0) {
                planes[(wave - 1) * 128 + r] = sa;
                planes[(wave - 1) * 128 + 64 + r] = sb;
            }
            __syncthreads();
            if (wave != 0) continue;
            if (grp == 0)
                for (int w = 0; w < NP - 1; ++w) {
                    const double4 xa = planes[w * 128 + r], xb = planes[w * 128 + 64 + r];
                    sa.x += xa.x; sa.y += xa.y; sa.z += xa.z; sa.w += xa.w;
                    sb.x += xb.x; sb.y += xb.y; sb.z += xb.z; sb.w += xb.w;
                }
        }
        if (grp == 0) {
            emit(t0 + tc + r, sa);
            if (hasb) emit(t0 + tc + r + G, sb);
        }
    }
}

template <typename T, int NP>
static void p2p_go(unsigned grid, int L, uint32_t per, const void *src, const uint32_t *start, double4 *out,
                   const Combine *fuse, hipStream_t st) {
    using V = typename V4<T>::type;
    const Combine c = fuse ? *fuse : Combine{};
    if (!fuse)
        k_p2p<T, NP, 0><<<grid, 64 * NP, 0, st>>>(L, per, (const V *)src, start, out, c);
    else if (fuse->dtype == FMM_F64)
        k_p2p<T, NP, 2><<<grid, 64 * NP, 0, st>>>(L, per, (const V *)src, start, out, c);
    else
        k_p2p<T, NP, 1><<<grid, 64 * NP, 0, st>>>(L, per, (const V *)src, start, out, c);
}

hipError_t launch_p2p(int L, bool f64, const void *src, const uint32_t *start, double4 *out, const Combine *fuse,
                      hipStream_t st) {
    const uint32_t nleaf = 1u << (3 * L);
    const uint32_t per = (nleaf + 7) / 8;
    const unsigned grid = per * 8;
    // below 4 waves per SIMD with one wave per leaf, split the neighbours
    if (nleaf <= 4096) {
        if (f64)
            p2p_go<double, 3>(grid, L, per, src, start, out, fuse, st);
        else
            p2p_go<float, 3>(grid, L, per, src, start, out, fuse, st);
    } else {
        if (f64)
            p2p_go<double, 1>(grid, L, per, src, start, out, fuse, st);
        else
            p2p_go<float, 1>(grid, L, per, src, start, out, fuse, st);
    }
    return hipGetLastError();
}

}  // namespace fmm

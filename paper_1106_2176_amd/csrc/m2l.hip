// m2l.hip -- multipole-to-local translation on the matrix cores.
//
// M2L is the one dense contraction of the method (Sec. 3.1: P2P and M2L are
// the two dominant kernels; Sec. 5: M2L runs at every level with no
// synchronisation between levels).  With level-independent operators
// (see opgen.cpp), a target box t of child class k (the parity of its
// coordinates) receives
//     L(t) = sum_{d in D_k} F_d M(t + d),
// over the 189 source offsets d of its class (children of the parent's
// neighbours that are not neighbours).  Grouping by offset turns this into
// one GEMM per (level, class): rows = p^2 local coefficients (padded to
// 16-row MFMA tiles), columns = the targets of the class, and the K
// dimension the concatenation over the 189 offsets of the p^2 multipole
// coefficients of the shifted source box.  Sources come from a zero-padded
// grid with a 3-box halo, so t + d is always a valid address and the shift
// of every column is the same constant for a given offset.
//
// Mixed form: operands stored in FP32 and split on the fly into bf16 parts
// x = x0 + x1 (+ x2); the products x_i y_j with i + j < parts are
// accumulated by v_mfma_f32_16x16x32_bf16 in FP32 and merged into FP64
// accumulators every 256 K terms.
// Plain form: v_mfma_f64_16x16x4_f64.
// MFMA operand layout (16 x 16 tiles, 64 lanes): A lane l holds row l%16,
// K-group l/16; B lane l holds column l%16, K-group l/16.  Results: for the
// bf16 instruction lane l holds rows 4(l/16) .. 4(l/16)+3 of column l%16; for
// the FP64 instruction lane l, item i holds row l/16 + 4i of column l%16
// (both layouts measured on gfx950).
#include "kernels.hpp"

namespace fmm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline int64_t unpack_delta(int e, int64_t G) {
    const int dx = (e & 15) - 4, dy = ((e >> 4) & 15) - 4, dz = ((e >> 8) & 15) - 4;
    return (int64_t)dx + G * ((int64_t)dy + G * (int64_t)dz);
}

// Work decomposition (both kernels): a block of four waves owns a tile of 128
// targets of one class (128 consecutive parents in Morton order) and all p^2
// output rows; each wave owns 32 targets (two 16-column MFMA blocks).  Every
// level runs in the same launch (the levels are independent): a block finds
// its level from the per-level block offsets.  Per block, the operator id and
// the source shift of each of the 189 offsets of its class are first cached
// in LDS; the operator rows of the current K-chunk are staged in LDS (double
// buffered, loaded by all waves) and the shifted source multipoles of the next
// chunk are prefetched into registers while the current chunk runs on the
// matrix cores.  Blocks are dealt round-robin to the 8 XCDs; when the level is
// large enough each XCD gets the tiles of one Morton octant of the parent
// grid, so its L2 holds that octant's sources.
constexpr int kTile = 128;
constexpr int kMaxLev = FMM_MAX_LEVEL + 1;

struct M2LLevels {
    int nlev;
    int level[kMaxLev];
    int64_t block0[kMaxLev + 1];  // first block of each level
    const void *B[kMaxLev];       // padded operand grid of the level
    void *L[kMaxLev];             // local expansions of the level
    int out_f64[kMaxLev];
};

struct M2LBlock {
    int li;         // index into M2LLevels
    int l;          // level
    int k;          // child class
    int64_t pbase;  // first parent (Morton) of the tile
};

__device__ inline M2LBlock m2l_block(const M2LLevels &ls) {
    M2LBlock t;
    const int64_t b = blockIdx.x;
    int li = 0;
    while (li + 1 < ls.nlev && b >= ls.block0[li + 1]) ++li;
    t.li = li;
    t.l = ls.level[li];
    const int64_t h = (int64_t)1 << (t.l - 1), npar = h * h * h;
    const int64_t lb = b - ls.block0[li];
    if (npar >= 8 * kTile) {
        const int64_t xcd = lb & 7, j = lb >> 3;
        t.k = (int)(j & 7);
        t.pbase = xcd * (npar >> 3) + (j >> 3) * kTile;
    } else {
        t.k = (int)(lb & 7);
        t.pbase = (lb >> 3) * kTile;
    }
    return t;
}

// bf16 parts of FP32 values: part 0 = RNE(x), part i = RNE of the remainder
__device__ inline uint32_t bf16_pack2(float a, float b, float &ra, float &rb) {
    uint32_t ua = __float_as_uint(a), ub = __float_as_uint(b);
    ua += 0x7fffu + ((ua >> 16) & 1u);
    ub += 0x7fffu + ((ub >> 16) & 1u);
    ua &= 0xffff0000u;
    ub &= 0xffff0000u;
    ra = a - __uint_as_float(ua);
    rb = b - __uint_as_float(ub);
    return (ua >> 16) | ub;
}

template <int NSPLIT>
__device__ inline void split8(const float4 lo4, const float4 hi4, bf16x8 (&out)[NSPLIT]) {
    float v[8] = {lo4.x, lo4.y, lo4.z, lo4.w, hi4.x, hi4.y, hi4.z, hi4.w};
#pragma unroll
    for (int s = 0; s < NSPLIT; ++s) {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = bf16_pack2(v[2 * i], v[2 * i + 1], v[2 * i], v[2 * i + 1]);
        out[s] = __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
    }
}

// Mixed form.  Operators and source multipoles are stored in FP32 and split
// into NSPLIT bf16 parts on the fly (operators while being staged into LDS,
// multipoles in registers).  Block = 8 waves = 128 targets; each wave owns
// one 16-target column block and all row tiles.
template <int NSPLIT, int RT>
__global__ __launch_bounds__(512) void k_m2l_bf16(int P, M2LLevels ls, const float *__restrict__ A,
                                                  const int2 *__restrict__ cls) {
    constexpr int R = RT * 16;
    constexpr int KP = 4;                      // pieces of 8 K per chunk (one MFMA K-step)
    constexpr int ROWP = 8 * KP + 8;           // LDS row pitch in bf16
    constexpr int NEL = R * 8 * KP;            // FP32 operator values per chunk
    constexpr int EPT = (NEL / 4 + 511) / 512; // float4 per thread
    __shared__ __align__(16) uint16_t As[2][NSPLIT][R][ROWP];
    __shared__ int sA[kOffsetsPerClass], sB[kOffsetsPerClass];

    const M2LBlock tb = m2l_block(ls);
    const int l = tb.l, k = tb.k;
    const float *__restrict__ B = (const float *)ls.B[tb.li];
    const int S = coef_stride(P), PPO = S / 8, P2 = P * P;
    const int n = 1 << l, h = n >> 1;
    const int64_t G = n + 6;
    const int64_t npar = (int64_t)h * h * h;
    const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4, col = lane & 15;

    for (int i = tid; i < kOffsetsPerClass; i += 512) {
        const int2 e = cls[k * kOffsetsPerClass + i];
        sA[i] = e.y * R * S;
        sB[i] = (int)unpack_delta(e.x, G) * S;
    }
    const int64_t pid = tb.pbase + wave * 16 + col;
    const bool cvalid = pid < npar;
    int64_t tpad, trow;
    {
        const uint32_t pc = cvalid ? (uint32_t)pid : 0u;
        const int64_t tx = 2 * (int64_t)compact3(pc) + kx, ty = 2 * (int64_t)compact3(pc >> 1) + ky,
                      tz = 2 * (int64_t)compact3(pc >> 2) + kz;
        tpad = ((tx + 3) + G * ((ty + 3) + G * (tz + 3))) * S;
        trow = tx + (int64_t)n * (ty + (int64_t)n * tz);
    }
    __syncthreads();
    const int NPC = kOffsetsPerClass * PPO;
    const int NCH = (NPC + KP - 1) / KP;

    // Operator chunk kc: R rows x 32 K as float4 quads (quad e -> row e/8,
    // quad e%8); multipole chunk kc: 8 FP32 values of piece 4 kc + q.  Loads
    // run D chunks ahead of the MFMAs through a ring of register stages.
    // Every load is issued unconditionally (so the compiler can keep the ring
    // in flight): pieces past the end read the zero operator appended to the
    // tables (id 316) and the all-zero halo box at the start of the grid.
    constexpr int D = 6;
    const int zeroA = kNumOffsets * R * S;
    const int NCHP = (NCH + D - 1) / D * D;
    float4 ar[D][EPT];
    float4 bl[D], bh[D];
    auto load_stage = [&](int kc, float4 (&a)[EPT], float4 &b0, float4 &b1) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = min(tid + 512 * i, NEL / 4 - 1);
            const int row = e >> 3, qd = e & 7;
            const int g = KP * kc + (qd >> 1);
            const int slot = min(g / PPO, kOffsetsPerClass - 1), cp = g - (g / PPO) * PPO;
            const int base = g < NPC ? sA[slot] : zeroA;
            a[i] = *(const float4 *)(A + base + row * S + 8 * cp + 4 * (qd & 1));
        }
        const int g = KP * kc + q;
        const int slot = min(g / PPO, kOffsetsPerClass - 1), cp = g - (g / PPO) * PPO;
        const float *src = g < NPC ? B + tpad + sB[slot] + 8 * cp : B;
        b0 = *(const float4 *)src;
        b1 = *(const float4 *)(src + 4);
    };
    auto store_a = [&](int buf, const float4 (&a)[EPT]) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + 512 * i;
            if (e < NEL / 4) {
                const int row = e >> 3, qd = e & 7;
                float v[4] = {a[i].x, a[i].y, a[i].z, a[i].w};
#pragma unroll
                for (int s = 0; s < NSPLIT; ++s) {
                    const uint32_t w0 = bf16_pack2(v[0], v[1], v[0], v[1]);
                    const uint32_t w1 = bf16_pack2(v[2], v[3], v[2], v[3]);
                    *(uint2 *)&As[buf][s][row][4 * qd] = make_uint2(w0, w1);
                }
            }
        }
    };

    f32x4 acc[RT];
    f64x4 acc64[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        acc[r] = f32x4{0, 0, 0, 0};
        acc64[r] = f64x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int d = 0; d < D; ++d) load_stage(d, ar[d], bl[d], bh[d]);
    store_a(0, ar[0]);
    __syncthreads();
    for (int kc0 = 0; kc0 < NCHP; kc0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int kc = kc0 + d;
            store_a((kc + 1) & 1, ar[(d + 1) % D]);
            bf16x8 bf[NSPLIT];
            split8<NSPLIT>(bl[d], bh[d], bf);
            const int cur = kc & 1;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                bf16x8 af[NSPLIT];
#pragma unroll
                for (int s = 0; s < NSPLIT; ++s) af[s] = *(const bf16x8 *)&As[cur][s][16 * r + col][8 * q];
#pragma unroll
                for (int i = 0; i < NSPLIT; ++i)
#pragma unroll
                    for (int j = 0; i + j < NSPLIT; ++j)
                        acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[r], 0, 0, 0);
            }
            load_stage(kc + D, ar[d], bl[d], bh[d]);
            if ((kc & 7) == 7) {  // merge every 256 K terms
#pragma unroll
                for (int r = 0; r < RT; ++r) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc64[r][i] += (double)acc[r][i];
                    acc[r] = f32x4{0, 0, 0, 0};
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc64[r][i] += (double)acc[r][i];
    if (!cvalid) return;
    void *Lout = ls.L[tb.li];
    const int out_f64 = ls.out_f64[tb.li];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * r + 4 * q + i;
            if (row < P2) {
                if (out_f64)
                    ((double *)Lout)[trow * S + row] = acc64[r][i];
                else
                    ((float *)Lout)[trow * S + row] = (float)acc64[r][i];
            }
        }
}

// FP64: K-chunks of 16 (four MFMA K-steps); lane group q takes K index
// 16 kc + 4 j + q in step j.
template <int RT>
__global__ __launch_bounds__(256) void k_m2l_f64(int P, M2LLevels ls, const double *__restrict__ A,
                                                 const int2 *__restrict__ cls) {
    constexpr int NB = 2, R = RT * 16, KC = 16, ROWP = KC + 1;
    constexpr int NEL = R * KC;
    constexpr int EPT = (NEL + 255) / 256;
    __shared__ double As[2][R][ROWP];
    __shared__ int sA[kOffsetsPerClass], sB[kOffsetsPerClass];

    const M2LBlock tb = m2l_block(ls);
    const int l = tb.l, k = tb.k;
    const double *__restrict__ B = (const double *)ls.B[tb.li];
    const int S = coef_stride(P), P2 = P * P;
    const int n = 1 << l, h = n >> 1;
    const int64_t G = n + 6;
    const int64_t npar = (int64_t)h * h * h;
    const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4, col = lane & 15;

    for (int i = tid; i < kOffsetsPerClass; i += 256) {
        const int2 e = cls[k * kOffsetsPerClass + i];
        sA[i] = e.y * R * S;
        sB[i] = (int)unpack_delta(e.x, G) * S;
    }
    int64_t tpad[NB], trow[NB];
    bool cvalid[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int64_t pid = tb.pbase + wave * NB * 16 + b * 16 + col;
        cvalid[b] = pid < npar;
        const uint32_t pc = cvalid[b] ? (uint32_t)pid : 0u;
        const int64_t tx = 2 * (int64_t)compact3(pc) + kx, ty = 2 * (int64_t)compact3(pc >> 1) + ky,
                      tz = 2 * (int64_t)compact3(pc >> 2) + kz;
        tpad[b] = ((tx + 3) + G * ((ty + 3) + G * (tz + 3))) * S;
        trow[b] = tx + (int64_t)n * (ty + (int64_t)n * tz);
    }
    __syncthreads();
    const int NK = kOffsetsPerClass * P2;
    const int NCH = (NK + KC - 1) / KC;

    double areg[EPT];
    auto load_a = [&](int kc) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + 256 * i;
            double v = 0.0;
            if (e < NEL) {
                const int row = e / KC, kk = e - row * KC;
                const int g = KC * kc + kk;
                if (g < NK) {
                    const int slot = g / P2, c = g - slot * P2;
                    v = A[sA[slot] + row * S + c];
                }
            }
            areg[i] = v;
        }
    };
    auto store_a = [&](int buf) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + 256 * i;
            if (e < NEL) {
                const int row = e / KC, kk = e - row * KC;
                As[buf][row][kk] = areg[i];
            }
        }
    };
    double bcur[4][NB], bnext[4][NB];
    auto load_b = [&](int kc, double (&dst)[4][NB]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int g = KC * kc + 4 * j + q;
            if (g < NK) {
                const int slot = g / P2, c = g - slot * P2;
                const int64_t off = sB[slot] + c;
#pragma unroll
                for (int b = 0; b < NB; ++b) dst[j][b] = B[tpad[b] + off];
            } else {
#pragma unroll
                for (int b = 0; b < NB; ++b) dst[j][b] = 0.0;
            }
        }
    };
    f64x4 acc[RT][NB];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[r][b] = f64x4{0, 0, 0, 0};

    load_a(0);
    store_a(0);
    load_b(0, bcur);
    __syncthreads();
    int cur = 0;
    for (int kc = 0; kc < NCH; ++kc) {
        const bool more = kc + 1 < NCH;
        if (more) {
            load_a(kc + 1);
            load_b(kc + 1, bnext);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const double av = As[cur][16 * r + col][4 * j + q];
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[r][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bcur[j][b], acc[r][b], 0, 0, 0);
            }
        if (more) store_a(cur ^ 1);
        __syncthreads();
        cur ^= 1;
        if (more) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int b = 0; b < NB; ++b) bcur[j][b] = bnext[j][b];
        }
    }
    double *Lout = (double *)ls.L[tb.li];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (!cvalid[b]) continue;
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // FP64 MFMA result layout: lane l, item i holds row l/16 + 4 i
                const int row = 16 * r + q + 4 * i;
                if (row < P2) Lout[trow[b] * S + row] = acc[r][b][i];
            }
    }
}

static int64_t m2l_blocks(int l) {
    const int64_t h = (int64_t)1 << (l - 1);
    const int64_t npar = h * h * h;
    return 8 * ((npar + kTile - 1) / kTile);
}

hipError_t launch_m2l(int P, int L, bool f64, int nsplit, void *const *B, void *const *Lc,
                      const int *out_f64, const void *A, size_t astride, const int2 *cls,
                      hipStream_t st) {
    if (L < 2) return hipSuccess;
    M2LLevels ls{};
    ls.nlev = L - 1;
    int64_t nb = 0;
    for (int i = 0; i < ls.nlev; ++i) {
        const int l = L - i;  // the largest level first: its blocks start earliest
        ls.level[i] = l;
        ls.block0[i] = nb;
        ls.B[i] = B[l];
        ls.L[i] = Lc[l];
        ls.out_f64[i] = out_f64[l];
        nb += m2l_blocks(l);
    }
    ls.block0[ls.nlev] = nb;
    const int RT = m2l_rows(P) / 16;
    if (f64) {
        switch (RT) {
#define CASE(RR) \
    case RR: k_m2l_f64<RR><<<(unsigned)nb, 256, 0, st>>>(P, ls, (const double *)A, cls); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
            CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (RT) {
#define CASE(RR)                                                                                        \
    case RR:                                                                                            \
        if (nsplit == 3)                                                                                \
            k_m2l_bf16<3, RR><<<(unsigned)nb, 512, 0, st>>>(P, ls, (const float *)A, cls);        \
        else                                                                                            \
            k_m2l_bf16<2, RR><<<(unsigned)nb, 512, 0, st>>>(P, ls, (const float *)A, cls);        \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
            CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace fmm

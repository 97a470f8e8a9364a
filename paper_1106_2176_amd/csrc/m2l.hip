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
// Mixed form: operands split into bf16 parts x = x0 + x1 (+ x2), each part
// the round-to-nearest-even bf16 of what the previous parts leave
// (operators once at set-up, multipoles in registers from FP32); the
// products x_i y_j with i + j < parts are accumulated by
// v_mfma_f32_16x16x32_bf16 in FP32 and merged into FP64 accumulators every
// 256 K terms.  Plain form: v_mfma_f64_16x16x4_f64.
// MFMA operand layout (16 x 16 tiles, 64 lanes): A lane l holds row l%16,
// K-group l/16; B lane l holds column l%16, K-group l/16.  Results: for the
// bf16 instruction lane l holds rows 4(l/16) .. 4(l/16)+3 of column l%16; for
// the FP64 instruction lane l, item i holds row l/16 + 4i of column l%16
// (both layouts measured on gfx950).
#include <algorithm>
#include <map>
#include <mutex>
#include <queue>
#include <tuple>
#include <vector>

#include "kernels.hpp"

namespace fmm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline int64_t unpack_delta(int e, int64_t G) {
    const int dx = (e & 15) - 4, dy = ((e >> 4) & 15) - 4, dz = ((e >> 8) & 15) - 4;
    return (int64_t)dx + G * ((int64_t)dy + G * (int64_t)dz);
}

// ------------------------------------------------------------ work plan
// A tile is 128 targets of one class at one level (128 consecutive parents
// in Morton order) and all p^2 output rows; a block owns one tile: eight
// waves of 16 targets each (two waves per SIMD, so that one wave's MFMAs run
// while the other waits on a load), or, where that operator ring does not
// fit in LDS, four waves of 32 targets (two 16-column MFMA blocks).  Every level runs
// in the same launch.  A tile's K range (the 189 offsets) may be cut into
// `nsplit` parts, each a block of its own, so that the small levels fill the
// chip after the largest level's tiles: the parts write FP64 partial sums
// and a fix-up kernel adds them in part order (deterministic, no atomics).
// Blocks are dealt round-robin to the 8 XCDs; when a level is large enough
// each XCD gets the tiles of one Morton octant of the parent grid (its L2
// holds that octant's sources), and consecutive blocks of an XCD cycle
// through the 8 classes, so the blocks running at one time on an XCD read
// the same operator stream roughly in step.
constexpr int kTile = 128;
constexpr int kMaxLev = FMM_MAX_LEVEL + 1;

struct M2LPlan {
    int nlev;
    int level[kMaxLev];
    int64_t unit0[kMaxLev + 1];  // first block of each level
    int64_t ntile[kMaxLev];      // tiles of the level (8 classes)
    int nsplit[kMaxLev];         // K parts per tile
    int64_t part0[kMaxLev];      // first partial slot of the level
    const void *B[kMaxLev];      // padded operand grid of the level
    void *L[kMaxLev];            // local expansions of the level
    int out_f64[kMaxLev];
    int64_t fix0[kMaxLev + 1];   // first fix-up block of each level
    // binary16 encoding: per-level maxima (by level) from which the operand
    // scale follows, and the output scale of each row
    const uint32_t *lmax;
    const float *oscale;
};

struct M2LUnit {
    int li;         // index into M2LPlan
    int l;          // level
    int k;          // child class
    int part;       // K part
    int64_t tile;   // tile within the level
    int64_t pbase;  // first parent (Morton) of the tile
};

// Uniform selection from the per-level kernel-argument arrays (an unrolled
// select chain: indexing them with a runtime value would copy the whole
// argument struct to scratch memory).
template <typename T, int N>
__device__ inline T pick(const T (&a)[N], int i) {
    T v = a[0];
#pragma unroll
    for (int j = 1; j < N; ++j)
        if (i == j) v = a[j];
    return v;
}

__device__ inline int find_level(const int64_t (&first)[kMaxLev + 1], int nlev, int64_t b) {
    int li = 0;
#pragma unroll
    for (int j = 1; j < kMaxLev; ++j)
        if (j < nlev && b >= first[j]) li = j;
    return li;
}

__device__ inline void tile_place(int l, int64_t lt, int &k, int64_t &pbase) {
    const int64_t h = (int64_t)1 << (l - 1), npar = h * h * h;
    if (npar >= 8 * kTile) {
        const int64_t xcd = lt & 7, j = lt >> 3;
        k = (int)(j & 7);
        pbase = xcd * (npar >> 3) + (j >> 3) * kTile;
    } else {
        k = (int)(lt & 7);
        pbase = (lt >> 3) * kTile;
    }
}

__device__ inline M2LUnit m2l_unit(const M2LPlan &pl) {
    M2LUnit u;
    const int64_t b = blockIdx.x;
    u.li = find_level(pl.unit0, pl.nlev, b);
    u.l = pick(pl.level, u.li);
    const int64_t nt = pick(pl.ntile, u.li);
    const int64_t ul = b - pick(pl.unit0, u.li);
    u.part = (int)(ul / nt);
    u.tile = ul - (int64_t)u.part * nt;
    tile_place(u.l, u.tile, u.k, u.pbase);
    return u;
}

// target box of parent `pid` in class k: padded-grid offset and output row
__device__ inline void target_of(int64_t pid, int k, int n, int64_t G, int S, int64_t &tpad,
                                 int64_t &trow) {
    const uint32_t pc = (uint32_t)pid;
    const int64_t tx = 2 * (int64_t)compact3(pc) + (k & 1), ty = 2 * (int64_t)compact3(pc >> 1) + ((k >> 1) & 1),
                  tz = 2 * (int64_t)compact3(pc >> 2) + (k >> 2);
    tpad = ((tx + 3) + G * ((ty + 3) + G * (tz + 3))) * S;
    trow = tx + (int64_t)n * (ty + (int64_t)n * tz);
}

// ------------------------------------------------------------ mixed form
// gfx950 copies global memory straight into LDS: each lane's 16 bytes land
// at (LDS base + 16 * lane); the base must be uniform over the wave.
__device__ __forceinline__ void dma16(const void *g, void *lds) {
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)g,
                                     (void __attribute__((address_space(3))) *)lds, 16, 0, 0);
}

// s_waitcnt with vmcnt = N (expcnt, lgkmcnt left at their maxima)
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit counter");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Workgroup barrier with this wave's LDS reads complete.  Written as one asm
// statement with a memory clobber so that the compiler moves no memory
// access across it and adds no wait of its own for the global loads still
// in flight (the operator ring is synchronised by the explicit vmcnt waits).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// bf16 parts of 8 FP32 values (one MFMA operand piece), hardware
// v_cvt_pk_bf16_f32 (round to nearest even) on what the previous parts leave
template <int NSPLIT>
__device__ __forceinline__ void split8(const float4 lo4, const float4 hi4, bf16x8 (&out)[NSPLIT]) {
    f32x2_t v[4] = {{lo4.x, lo4.y}, {lo4.z, lo4.w}, {hi4.x, hi4.y}, {hi4.z, hi4.w}};
#pragma unroll
    for (int s = 0; s < NSPLIT; ++s) {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            w[i] = __builtin_bit_cast(uint32_t, __builtin_convertvector(v[i], bf16x2_t));
            if (s + 1 < NSPLIT) {
                v[i].x -= __uint_as_float(w[i] << 16);
                v[i].y -= __uint_as_float(w[i] & 0xffff0000u);
            }
        }
        out[s] = __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
    }
}

// Multipole operand parts of one 8-wide piece: the bf16 split of the FP32
// values, or (binary16 encoding, H) the two parts the pack kernel stored,
// hi8 in the piece's first 16 bytes and lo8 in the second.
template <int NSPLIT, bool H>
__device__ __forceinline__ void b_parts(const float4 a, const float4 b, bf16x8 (&out)[NSPLIT]) {
    if constexpr (H) {
        static_assert(NSPLIT == 2, "the binary16 encoding has two parts");
        out[0] = __builtin_bit_cast(bf16x8, a);
        out[1] = __builtin_bit_cast(bf16x8, b);
    } else {
        split8<NSPLIT>(a, b, out);
    }
}

// One 16x16x32 product on the matrix cores, bf16 or binary16 operands
// (both held as 16-byte fragments), FP32 accumulation.
template <bool H>
__device__ __forceinline__ f32x4 mfma32(const bf16x8 a, const bf16x8 b, const f32x4 c) {
    if constexpr (H)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                       __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

template <int NSPLIT, int P, int NW>
struct MixCfg {
    static constexpr int P2 = P * P, S = coef_stride(P), PPO = S / 8;
    static constexpr int RT = m2l_rows(P) / 16, R = RT * 16;
    static constexpr int NB = 8 / NW;                // 16-column blocks per wave (128 columns per tile)
    static constexpr int NCHK = NSPLIT * RT;         // 1 KB operator chunks per K-step
    static constexpr int CPW = (NCHK + NW - 1) / NW; // chunks loaded per wave
    static constexpr int STAGE = NW * CPW;           // chunk slots per ring stage
    // operator ring stages in LDS (4; deeper rings, 6 or 8 where LDS holds
    // them, measured no faster and spill registers at p = 10); multipole ring
    // stages in registers: 4 (8 measured no faster with eight waves).  The
    // step loop is unrolled over both rings (UNROLL = lcm) with an FP64 merge
    // every MERGE <= 8 steps.
    static constexpr int NA = 4;
    static constexpr int D = 4;
    static constexpr int UNROLL = NA == 6 ? 12 : 8;
    static constexpr int MERGE = NA == 6 ? 6 : 8;
    static constexpr int NBL = NB * 2;               // multipole loads per K-step
    // A fragments read one step ahead (step) while the two steps' fragments
    // and the accumulators fit two waves per SIMD without spilling (up to
    // p = 12 with two parts, 11 with three), else during their own step,
    // one split part at a time (step8)
    static constexpr bool PIPE = NW != 8 || 8 * NSPLIT * RT + 12 * RT <= 288;
    // loads this wave issues after the operator chunks it waits for at the
    // top of step kc (those of step kc + 1 with PIPE, else of step kc, issued
    // NA - 1 steps earlier either way): the multipole loads of that step and
    // everything of the NA - 2 steps between
    static constexpr int VMW = NBL + (NA - 2) * (CPW + NBL);
    static constexpr int NPC = kOffsetsPerClass * PPO;  // K pieces of a class
    static constexpr int NCH = ((NPC + 3) / 4 + UNROLL - 1) / UNROLL * UNROLL;  // K-steps, padded
    static_assert(VMW < 64, "vmcnt range");
};

// Operators: pre-split bf16 parts [part][317][R/16][S/8][16][8] (operator
// 316 is zero); multipoles: the FP32 padded grid [G^3][S] (box 0 is a halo
// box, all zero).  K-step kc covers the 4 pieces (8 K each) 4 kc .. 4 kc + 3
// of the class's concatenated K range; a lane's piece is g = 4 kc + q.  The
// operator chunk (part s, row tile r) of a K-step is copied to LDS in MFMA
// fragment order (lane L = (g4, c): row 16 r + c, piece 4 kc + g4): one
// contiguous kilobyte of the operator table unless the 4 pieces straddle two
// offsets, and one contiguous kilobyte of LDS for the wave's fragment read.
// All loads are unconditional: pieces past the end read the zero operator
// and the zero box.
template <int NSPLIT, int P, int NW, bool H>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4))) void k_m2l_bf16(
    M2LPlan pl, const uint16_t *__restrict__ A, size_t astride, const int2 *__restrict__ cls,
    double *__restrict__ partial) {
    using C = MixCfg<NSPLIT, P, NW>;
    static_assert(C::NA * C::STAGE <= 150, "LDS");
    constexpr int P2 = C::P2, S = C::S, PPO = C::PPO, RT = C::RT, R = C::R, NB = C::NB;
    constexpr int NCHK = C::NCHK, CPW = C::CPW, STAGE = C::STAGE, NA = C::NA, D = C::D;
    constexpr int NPC = C::NPC, NCH = C::NCH, UNROLL = C::UNROLL, MERGE = C::MERGE;
    // one LDS array per ring stage (arrays of stages the ring does not use
    // are never referenced and take no space)
    __shared__ __align__(16) uint4 ring0[STAGE * 64];
    __shared__ __align__(16) uint4 ring1[STAGE * 64];
    __shared__ __align__(16) uint4 ring2[STAGE * 64];
    __shared__ __align__(16) uint4 ring3[STAGE * 64];
    __shared__ __align__(16) uint4 ring4[STAGE * 64];
    __shared__ __align__(16) uint4 ring5[STAGE * 64];
    __shared__ __align__(16) uint4 ring6[STAGE * 64];
    __shared__ __align__(16) uint4 ring7[STAGE * 64];
    auto stage = [&](auto ic) __attribute__((always_inline)) -> uint4 * {
        constexpr int i = decltype(ic)::value % NA;
        if constexpr (i == 0) return ring0;
        else if constexpr (i == 1) return ring1;
        else if constexpr (i == 2) return ring2;
        else if constexpr (i == 3) return ring3;
        else if constexpr (i == 4) return ring4;
        else if constexpr (i == 5) return ring5;
        else if constexpr (i == 6) return ring6;
        else return ring7;
    };
    // per offset slot: operator base and source shift; slot 189 (pieces past
    // the end) holds the zero operator
    __shared__ int sA[kOffsetsPerClass + 1], sB[kOffsetsPerClass + 1];

    const M2LUnit u = m2l_unit(pl);
    const int l = u.l, k = u.k;
    const float *__restrict__ B = (const float *)pick(pl.B, u.li);
    const int nsplit = pick(pl.nsplit, u.li);
    const int n = 1 << l, h = n >> 1;
    const int64_t G = n + 6;
    const int64_t npar = (int64_t)h * h * h;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = lane >> 4, col = lane & 15;
    // K range of this part, in whole unrolled groups of steps
    const int kbeg = (int)((int64_t)u.part * (NCH / UNROLL) / nsplit) * UNROLL;
    const int kend = (int)((int64_t)(u.part + 1) * (NCH / UNROLL) / nsplit) * UNROLL;
    for (int i = tid; i <= kOffsetsPerClass; i += 64 * NW) {
        if (i == kOffsetsPerClass) {
            sA[i] = kNumOffsets * R * S;
            sB[i] = 0;
        } else {
            const int2 e = cls[k * kOffsetsPerClass + i];
            sA[i] = e.y * R * S;
            sB[i] = (int)unpack_delta(e.x, G) * S;
        }
    }
    int64_t tpad[NB], trow[NB];
    bool cvalid[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int64_t pid = u.pbase + wave * 16 * NB + b * 16 + col;
        cvalid[b] = pid < npar;
        target_of(cvalid[b] ? pid : 0, k, n, G, S, tpad[b], trow[b]);
    }
    __syncthreads();

    // per lane and K-step: operator base + piece offset, multipole offset
    // (table reads are unconditional: a branch here would split the step
    // into basic blocks)
    auto piece = [&](int kc, int &aoff, int &boff, bool &inb) __attribute__((always_inline)) {
        const int g = 4 * kc + q;
        inb = g < NPC;
        const int q8 = g / PPO;
        const int slot = inb ? q8 : kOffsetsPerClass;
        const int cp = inb ? g - q8 * PPO : 0;
        aoff = sA[slot] + 128 * cp + 8 * col;
        boff = sB[slot] + 8 * cp;
    };
    auto issue_a = [&](int kc, uint4 *stage) __attribute__((always_inline)) {
        int aoff, boff;
        bool inb;
        piece(kc, aoff, boff, inb);
#pragma unroll
        for (int i = 0; i < CPW; ++i) {
            const int ch = NW * i + wave;  // wave-uniform
            const int c0 = ch < NCHK ? ch : 0;
            const int sp = c0 / RT, r = c0 - sp * RT;
            dma16(A + sp * astride + aoff + 16 * r * S, stage + ch * 64);
        }
    };
    auto issue_b = [&](int kc, float4 (&bv)[NB][2]) __attribute__((always_inline)) {
        int aoff, boff;
        bool inb;
        piece(kc, aoff, boff, inb);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float *src = B + (inb ? tpad[b] + boff : 0);
            bv[b][0] = *(const float4 *)src;
            bv[b][1] = *(const float4 *)(src + 4);
        }
    };

    f32x4 acc[RT][NB];
    f64x4 acc64[RT][NB];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            acc[r][b] = f32x4{0, 0, 0, 0};
            acc64[r][b] = f64x4{0, 0, 0, 0};
        }

    // Pipeline: an NA-stage operator ring in LDS and a D-stage multipole ring
    // in registers.  At the top of step kc the A fragments and the bf16
    // parts of the multipoles of step kc are already in registers (read and
    // split during step kc - 1), so the matrix cores start right after the
    // barrier.  Step kc: wait until this wave's copies for step kc + 1 are in
    // LDS; barrier (everyone's are, and everyone has read stage kc); start
    // the copy of step kc + NA into stage kc; issue the MFMAs of step kc
    // while reading the A fragments of step kc + 1 and splitting its
    // multipoles; load the multipoles of step kc + D.  i (the step's
    // position in the unrolled group, hence both ring stages) is a
    // compile-time constant.
    auto read_a = [&](const uint4 *st, bf16x8 (&af)[RT][NSPLIT]) __attribute__((always_inline)) {
#pragma unroll
        for (int sp = 0; sp < NSPLIT; ++sp)
#pragma unroll
            for (int r = 0; r < RT; ++r)
                af[r][sp] = __builtin_bit_cast(bf16x8, st[(sp * RT + r) * 64 + lane]);
    };
    float4 bv[D][NB][2];
    bf16x8 af[RT][NSPLIT], bf[NB][NSPLIT];
    // Without PIPE each step's A fragments are read from its own stage
    // during the step, so the ring is one step shorter: step kc copies step
    // kc + NA - 1 into the stage of step kc - 1, which every wave has finished
    // reading by step kc's barrier.  Reading them a step ahead (PIPE) lets the
    // matrix products start right after the barrier: 2.3% faster at C2 and
    // C3 (p = 10), where waiting at every step for all of the step's
    // fragments had held them back.
    constexpr bool PIPE = C::PIPE;
    constexpr int PRE = PIPE ? NA : NA - 1;
    static_for<0, PRE>([&](auto ic) __attribute__((always_inline)) {
        issue_a(kbeg + decltype(ic)::value, stage(ic));
    });
#pragma unroll
    for (int d = 0; d < D; ++d) issue_b(kbeg + d, bv[d]);
    // Drain the prologue once: with loads from before the loop still pending
    // at the loop header, the compiler cannot tell them from the loop's own
    // and waits for every load in flight at each pass through the header.
    wait_vm<0>();
    lds_barrier();
    if constexpr (PIPE) read_a(stage(std::integral_constant<int, 0>{}), af);
#pragma unroll
    for (int b = 0; b < NB; ++b) b_parts<NSPLIT, H>(bv[0][b][0], bv[0][b][1], bf[b]);

    // A fragments of split part sp of a stage
    auto read_part = [&](const uint4 *st, int sp, bf16x8 (&ap)[RT]) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < RT; ++r) ap[r] = __builtin_bit_cast(bf16x8, st[(sp * RT + r) * 64 + lane]);
    };
    auto step8 = [&](int kc, auto dc) __attribute__((always_inline)) {
        constexpr int i = decltype(dc)::value;
        constexpr int d = i % D, dn = (i + 1) % D;
        const uint4 *const cur = stage(std::integral_constant<int, i>{});
        uint4 *const prev = stage(std::integral_constant<int, i + NA - 1>{});
        wait_vm<C::VMW>();  // this wave's operator chunks of step kc are in LDS
        lds_barrier();      // ... and everyone's; the stage of step kc - 1 is free
        issue_a(kc + NA - 1, prev);
        bf16x8 ap[2][RT], bn[NB][NSPLIT];
        read_part(cur, NSPLIT - 1, ap[0]);
#pragma unroll
        for (int b = 0; b < NB; ++b) b_parts<NSPLIT, H>(bv[dn][b][0], bv[dn][b][1], bn[b]);
        // A parts from the smallest; within a part, the small B parts first
        static_for<0, NSPLIT>([&](auto jc) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value, a = NSPLIT - 1 - j;
            if constexpr (j + 1 < NSPLIT) read_part(cur, a - 1, ap[(j + 1) & 1]);
#pragma unroll
            for (int t = NSPLIT - 1 - a; t >= 0; --t)
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[r][b] = mfma32<H>(ap[j & 1][r], bf[b][t], acc[r][b]);
        });
        issue_b(kc + D, bv[d]);
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int sp = 0; sp < NSPLIT; ++sp) bf[b][sp] = bn[b][sp];
    };

    auto step = [&](int kc, auto dc) __attribute__((always_inline)) {
        constexpr int i = decltype(dc)::value;
        constexpr int d = i % D, dn = (i + 1) % D;
        uint4 *const cur = stage(std::integral_constant<int, i>{});
        uint4 *const nxt = stage(std::integral_constant<int, i + 1>{});
        wait_vm<C::VMW>();  // this wave's operator chunks of step kc + 1 are in LDS
        lds_barrier();      // ... and everyone's; stage d has been read by all
        issue_a(kc + NA, cur);
        bf16x8 an[RT][NSPLIT], bn[NB][NSPLIT];
        read_a(nxt, an);
#pragma unroll
        for (int b = 0; b < NB; ++b) b_parts<NSPLIT, H>(bv[dn][b][0], bv[dn][b][1], bn[b]);
        // the small cross products first; consecutive MFMAs update different
        // accumulators (RT * NB independent chains)
#pragma unroll
        for (int t = NSPLIT - 1; t >= 0; --t)
#pragma unroll
            for (int a = 0; a <= t; ++a)
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[r][b] = mfma32<H>(af[r][a], bf[b][t - a], acc[r][b]);
        issue_b(kc + D, bv[d]);
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int sp = 0; sp < NSPLIT; ++sp) af[r][sp] = an[r][sp];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int sp = 0; sp < NSPLIT; ++sp) bf[b][sp] = bn[b][sp];
    };
    auto merge = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
#pragma unroll
                for (int i = 0; i < 4; ++i) acc64[r][b][i] += (double)acc[r][b][i];
                acc[r][b] = f32x4{0, 0, 0, 0};
            }
    };
    for (int kc = kbeg; kc < kend; kc += UNROLL) {
        static_for<0, UNROLL>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            if constexpr (PIPE)
                step(kc + i, ic);
            else
                step8(kc + i, ic);
            if constexpr ((i + 1) % MERGE == 0) merge();  // every MERGE * 32 <= 256 K terms
        });
    }
    wait_vm<0>();  // no copy into LDS outlives the block

    if constexpr (H) {
        // undo the encoding: row r of the result carries the table's row
        // scale a_r and the level's operand scale 2^e (powers of two)
        const int sh = -level_scale_exp(pl.lmax[l]);
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * r + 4 * q + i;
                const double f = row < P2 ? ldexp((double)pl.oscale[row], sh) : 0.0;
#pragma unroll
                for (int b = 0; b < NB; ++b) acc64[r][b][i] *= f;
            }
    }
    if (nsplit == 1) {
        void *Lout = pick(pl.L, u.li);
        const int out_f64 = pick(pl.out_f64, u.li);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (!cvalid[b]) continue;
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * r + 4 * q + i;
                    if (row < P2) {
                        if (out_f64)
                            ((double *)Lout)[trow[b] * S + row] = acc64[r][b][i];
                        else
                            ((float *)Lout)[trow[b] * S + row] = (float)acc64[r][b][i];
                    }
                }
        }
    } else {
        const int64_t slot = pick(pl.part0, u.li) + (int64_t)u.part * pick(pl.ntile, u.li) + u.tile;
        double *dst = partial + slot * kTile * P2;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * r + 4 * q + i;
                    if (row < P2) dst[(wave * 16 * NB + b * 16 + col) * P2 + row] = acc64[r][b][i];
                }
    }
}

// Sum of the K parts of a split tile, in part order.  One thread per output
// coefficient (tile, target column, row).
__global__ __launch_bounds__(256) void k_m2l_fixup(int P, M2LPlan pl, const double *__restrict__ partial,
                                                   int64_t total) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= total) return;
    const int P2 = P * P, S = coef_stride(P);
    const int64_t per_tile = (int64_t)kTile * P2;
    const int64_t ft = g / per_tile;
    const int e = (int)(g - ft * per_tile);
    const int li = find_level(pl.fix0, pl.nlev, ft);
    const int l = pick(pl.level, li), ns = pick(pl.nsplit, li);
    const int64_t nt = pick(pl.ntile, li), lt = ft - pick(pl.fix0, li);
    int k;
    int64_t pbase;
    tile_place(l, lt, k, pbase);
    const int n = 1 << l, h = n >> 1;
    const int64_t npar = (int64_t)h * h * h;
    const int c = e / P2, row = e - c * P2;
    const int64_t pid = pbase + c;
    if (pid >= npar) return;
    const double *src = partial + (pick(pl.part0, li) + lt) * per_tile + e;
    double v = 0.0;
    for (int j = 0; j < ns; ++j) v += src[(int64_t)j * nt * per_tile];
    int64_t tpad, trow;
    target_of(pid, k, n, n + 6, S, tpad, trow);
    if (pick(pl.out_f64, li))
        ((double *)pick(pl.L, li))[trow * S + row] = v;
    else
        ((float *)pick(pl.L, li))[trow * S + row] = (float)v;
}

// ------------------------------------------------------------ plain form
// FP64 operators [317][R][S] and the FP64 padded multipole grid.  K runs over
// the 189 offsets x S coefficients (entries past p^2 are zero in both), in
// chunks of 8 that never straddle an offset, so a chunk's operator and
// source shift are uniform over the block.  A chunk: R x 8 operator values
// staged in LDS (each thread loads EPT of them one chunk ahead, two register
// sets), then per wave RT x NB x 2 MFMAs (v_mfma_f64_16x16x4_f64, lane group
// q takes K index 4 j + q of the chunk).  Registers fit two blocks per CU up
// to p = 11 (one beyond).
template <int P, int WPE = (P <= 11 ? 2 : 1)>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void k_m2l_f64(
    M2LPlan pl, const double *__restrict__ A, const int2 *__restrict__ cls,
    double *__restrict__ partial) {
    constexpr int P2 = P * P, S = coef_stride(P), RT = m2l_rows(P) / 16, R = RT * 16;
    constexpr int NB = 2, KC = 8, ROWP = KC + 1, CPO = S / KC;  // chunks per offset
    constexpr int NEL = R * KC, EPT = (NEL + 255) / 256;
    constexpr int NCH = kOffsetsPerClass * CPO;
    __shared__ double As[2][R * ROWP];
    __shared__ int sA[kOffsetsPerClass], sB[kOffsetsPerClass];

    const M2LUnit u = m2l_unit(pl);
    const int l = u.l, k = u.k;
    const double *__restrict__ B = (const double *)pick(pl.B, u.li);
    const int n = 1 << l, h = n >> 1;
    const int64_t G = n + 6;
    const int64_t npar = (int64_t)h * h * h;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int nsplit = pick(pl.nsplit, u.li);
    const int kbeg = (int)((int64_t)u.part * NCH / nsplit);
    const int kend = (int)((int64_t)(u.part + 1) * NCH / nsplit);

    for (int i = tid; i < kOffsetsPerClass; i += 256) {
        const int2 e = cls[k * kOffsetsPerClass + i];
        sA[i] = e.y * R * S;
        sB[i] = (int)unpack_delta(e.x, G) * S;
    }
    int64_t tpad[NB], trow[NB];
    bool cvalid[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int64_t pid = u.pbase + wave * NB * 16 + b * 16 + col;
        cvalid[b] = pid < npar;
        target_of(cvalid[b] ? pid : 0, k, n, G, S, tpad[b], trow[b]);
    }
    __syncthreads();

    // this thread's elements of an A chunk: (row, kk) = (e / KC, e % KC)
    auto load_a = [&](int kc, double (&dst)[EPT]) __attribute__((always_inline)) {
        const int slot = kc / CPO, c0 = KC * (kc - slot * CPO);
        const double *a = A + sA[slot] + c0;
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + 256 * i;
            dst[i] = (NEL % 256 == 0 || e < NEL) ? a[(e / KC) * S + e % KC] : 0.0;
        }
    };
    auto store_a = [&](int buf, const double (&src)[EPT]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + 256 * i;
            if (NEL % 256 == 0 || e < NEL) As[buf][(e / KC) * ROWP + e % KC] = src[i];
        }
    };
    auto load_b = [&](int kc, double (&dst)[2][NB]) __attribute__((always_inline)) {
        const int slot = kc / CPO, c0 = KC * (kc - slot * CPO);
        const int64_t off = sB[slot] + c0 + q;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int b = 0; b < NB; ++b) dst[j][b] = B[tpad[b] + off + 4 * j];
    };

    f64x4 acc[RT][NB];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[r][b] = f64x4{0, 0, 0, 0};

    // step t = kc - kbeg: chunk kc is in LDS buffer t & 1, chunk kc + 1 in
    // register set t & 1 and chunk kc + 2 in the other (the last chunk is
    // loaded again past the end of the range)
    double ar[2][EPT], br[2][2][NB], bc[2][NB];
    load_a(kbeg, ar[0]);
    store_a(0, ar[0]);
    load_b(kbeg, bc);
    load_a(min(kbeg + 1, kend - 1), ar[0]);
    load_b(min(kbeg + 1, kend - 1), br[0]);
    load_a(min(kbeg + 2, kend - 1), ar[1]);
    load_b(min(kbeg + 2, kend - 1), br[1]);
    __syncthreads();
    auto chunk = [&](int kc, auto pc) __attribute__((always_inline)) {
        constexpr int ph = decltype(pc)::value;  // (kc - kbeg) & 1
        const double *as = As[ph];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const double av = as[(16 * r + col) * ROWP + 4 * j + q];
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[r][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bc[j][b], acc[r][b], 0, 0, 0);
            }
        store_a(ph ^ 1, ar[ph]);  // chunk kc + 1 into the other buffer, read by
                                  // every wave up to the last barrier
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int b = 0; b < NB; ++b) bc[j][b] = br[ph][j][b];
        load_a(min(kc + 3, kend - 1), ar[ph]);
        load_b(min(kc + 3, kend - 1), br[ph]);
        __syncthreads();
    };
    // a pair of chunks per pass keeps the parity a compile-time constant
    int kc = kbeg;
    for (; kc + 1 < kend; kc += 2) {
        chunk(kc, std::integral_constant<int, 0>{});
        chunk(kc + 1, std::integral_constant<int, 1>{});
    }
    if (kc < kend) chunk(kc, std::integral_constant<int, 0>{});

    // FP64 MFMA result layout: lane l, item i holds row l/16 + 4 i
    if (nsplit == 1) {
        double *Lout = (double *)pick(pl.L, u.li);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (!cvalid[b]) continue;
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * r + q + 4 * i;
                    if (row < P2) Lout[trow[b] * S + row] = acc[r][b][i];
                }
        }
    } else {
        const int64_t slot = pick(pl.part0, u.li) + (int64_t)u.part * pick(pl.ntile, u.li) + u.tile;
        double *dst = partial + slot * kTile * P2;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * r + q + 4 * i;
                    if (row < P2) dst[(wave * NB * 16 + b * 16 + col) * P2 + row] = acc[r][b][i];
                }
    }
}

// ------------------------------------------------ rotation-based M2L (FP64)
// O(p^3) per pair instead of O(p^4): the multipole of a source box is rotated
// into the frame whose z axis points along the offset (target minus source),
// translated along z, and the local expansion rotated back, F = D^T Tz D
// (the rotations of the paper's GPU code, Fig. 4).  D is block diagonal by
// degree (sum (2n+1)^2 entries), Tz by order and cosine/sine kind (sum over
// m of (p-m)^2 entries per kind).  A block takes kRotNT targets of one class
// at one level and walks the class's 189 offsets; per offset it stages the
// compact D and Tz and the targets' source multipoles in LDS and runs the
// three stages, each thread computing a row for kRotTT targets at a time;
// the rotated-back results accumulate in registers over all offsets.
constexpr int kRotNT = 16, kRotTT = 4, kRotThreads = 256;

struct RotPlan {
    int nlev;
    int level[kMaxLev];
    int64_t blk0[kMaxLev + 1];  // first block of each level
    const double *B[kMaxLev];   // FP64 padded multipole grid of the level
    double *L[kMaxLev];         // local expansions of the level
};

__device__ __forceinline__ int isqrt_small(int c) {
    int n = (int)sqrtf((float)c);
    while (n * n > c) --n;
    while ((n + 1) * (n + 1) <= c) ++n;
    return n;
}

template <int P>
__global__ __launch_bounds__(kRotThreads) void k_m2l_rot(RotPlan pl, const double *__restrict__ rot,
                                                        const double *__restrict__ tz,
                                                        const int2 *__restrict__ cls) {
    constexpr int P2 = P * P, S = coef_stride(P), ND = rot_size(P), NZ = tz_size(P);
    constexpr int NT = kRotNT, TT = kRotTT, NG = NT / TT, NI = P2 * NG;
    // LDS row pitch of the [coefficient][target] buffers: two doubles of
    // padding against bank conflicts, 16-byte rows kept aligned
    constexpr int NTP = NT + 2;
    constexpr int IPT = (NI + kRotThreads - 1) / kRotThreads;
    __shared__ double sD[ND], sT[NZ];
    __shared__ __align__(16) double sM[P2 * NTP], sX[P2 * NTP];  // [coefficient][target]
    __shared__ int64_t sTp[NT];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int li = find_level(pl.blk0, pl.nlev, b);
    const int l = pick(pl.level, li);
    const double *__restrict__ B = pick(pl.B, li);
    double *__restrict__ Lout = pick(pl.L, li);
    const int n = 1 << l, h = n >> 1;
    const int64_t G = n + 6, npar = (int64_t)h * h * h;
    const int64_t j = b - pick(pl.blk0, li);
    const int k = (int)(j & 7);
    const int64_t pbase = (j >> 3) * NT;
    if (tid < NT) {
        int64_t tp, tr;
        target_of(pbase + tid < npar ? pbase + tid : 0, k, n, G, S, tp, tr);
        sTp[tid] = tp;
    }
    double acc[IPT][TT];
#pragma unroll
    for (int it = 0; it < IPT; ++it)
#pragma unroll
        for (int t = 0; t < TT; ++t) acc[it][t] = 0.0;

    // The next offset's D, Tz and source multipoles are loaded into registers
    // while the current offset computes, and stored to LDS at the top of the
    // next step: the global-memory latency stays off the critical path.
    constexpr int LD = (ND + kRotThreads - 1) / kRotThreads, LZ = (NZ + kRotThreads - 1) / kRotThreads;
    constexpr int LM = (P2 * NT + kRotThreads - 1) / kRotThreads;
    double rD[LD], rZ[LZ], rM[LM];
    __syncthreads();  // sTp
    auto fetch = [&](int slot) __attribute__((always_inline)) {
        const int2 e = cls[k * kOffsetsPerClass + slot];
        const int64_t shift = unpack_delta(e.x, G) * S;
        const double *dsrc = rot + (size_t)e.y * ND, *tsrc = tz + (size_t)e.y * NZ;
#pragma unroll
        for (int u = 0; u < LD; ++u) {
            const int i = tid + u * kRotThreads;
            rD[u] = (ND % kRotThreads == 0 || i < ND) ? dsrc[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LZ; ++u) {
            const int i = tid + u * kRotThreads;
            rZ[u] = (NZ % kRotThreads == 0 || i < NZ) ? tsrc[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LM; ++u) {
            const int i = tid + u * kRotThreads;
            const int t = i / P2, c = i - t * P2;
            rM[u] = ((P2 * NT) % kRotThreads == 0 || i < P2 * NT) ? B[sTp[t] + shift + c] : 0.0;
        }
    };
    fetch(0);
    for (int slot = 0; slot < kOffsetsPerClass; ++slot) {
        __syncthreads();  // every thread is done with the previous offset's LDS
#pragma unroll
        for (int u = 0; u < LD; ++u) {
            const int i = tid + u * kRotThreads;
            if (ND % kRotThreads == 0 || i < ND) sD[i] = rD[u];
        }
#pragma unroll
        for (int u = 0; u < LZ; ++u) {
            const int i = tid + u * kRotThreads;
            if (NZ % kRotThreads == 0 || i < NZ) sT[i] = rZ[u];
        }
#pragma unroll
        for (int u = 0; u < LM; ++u) {
            const int i = tid + u * kRotThreads;
            const int t = i / P2, c = i - t * P2;
            if ((P2 * NT) % kRotThreads == 0 || i < P2 * NT) sM[c * NTP + t] = rM[u];
        }
        __syncthreads();
        if (slot + 1 < kOffsetsPerClass) fetch(slot + 1);
        // rotate: X = D M (within each degree block)
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const int item = tid + it * kRotThreads;
            if (NI % kRotThreads != 0 && item >= NI) break;
            const int r = item % P2, g = item / P2;
            const int dn = isqrt_small(r), rb = dn * dn, w = 2 * dn + 1;
            const double *drow = sD + rot_deg_off(dn) + (r - rb) * w;
            const double *mc = sM + rb * NTP + g * TT;
            double a4[TT] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int q = 0; q < w; ++q) {
                const double d = drow[q];
                const double2 m01 = *(const double2 *)(mc + q * NTP), m23 = *(const double2 *)(mc + q * NTP + 2);
                a4[0] += d * m01.x;
                a4[1] += d * m01.y;
                a4[2] += d * m23.x;
                a4[3] += d * m23.y;
            }
            double *xo = sX + r * NTP + g * TT;
            *(double2 *)xo = make_double2(a4[0], a4[1]);
            *(double2 *)(xo + 2) = make_double2(a4[2], a4[3]);
        }
        __syncthreads();
        // translate along z: Y = Tz X (within each order / kind), into sM
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const int item = tid + it * kRotThreads;
            if (NI % kRotThreads != 0 && item >= NI) break;
            const int r = item % P2, g = item / P2;
            const int kd = isqrt_small(r), rr = r - kd * kd;
            const int m = (rr + 1) >> 1, kind = (rr > 0 && !(rr & 1)) ? 1 : 0;
            const double *trow2 = sT + tz_off(P, m, kind) + (kd - m) * (P - m);
            double a4[TT] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int nn = m; nn < P; ++nn) {
                const int c = nn * nn + (m == 0 ? 0 : 2 * m - 1 + kind);
                const double tv = trow2[nn - m];
                const double *xc = sX + c * NTP + g * TT;
                const double2 x01 = *(const double2 *)xc, x23 = *(const double2 *)(xc + 2);
                a4[0] += tv * x01.x;
                a4[1] += tv * x01.y;
                a4[2] += tv * x23.x;
                a4[3] += tv * x23.y;
            }
            double *yo = sM + r * NTP + g * TT;
            *(double2 *)yo = make_double2(a4[0], a4[1]);
            *(double2 *)(yo + 2) = make_double2(a4[2], a4[3]);
        }
        __syncthreads();
        // rotate back and accumulate: acc += D^T Y
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const int item = tid + it * kRotThreads;
            if (NI % kRotThreads != 0 && item >= NI) break;
            const int r = item % P2, g = item / P2;
            const int dn = isqrt_small(r), rb = dn * dn, w = 2 * dn + 1;
            const double *dcol = sD + rot_deg_off(dn) + (r - rb);
            const double *yc = sM + rb * NTP + g * TT;
#pragma unroll 4
            for (int q = 0; q < w; ++q) {
                const double d = dcol[q * w];
                const double2 y01 = *(const double2 *)(yc + q * NTP), y23 = *(const double2 *)(yc + q * NTP + 2);
                acc[it][0] += d * y01.x;
                acc[it][1] += d * y01.y;
                acc[it][2] += d * y23.x;
                acc[it][3] += d * y23.y;
            }
        }
    }
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const int item = tid + it * kRotThreads;
        if (NI % kRotThreads != 0 && item >= NI) break;
        const int r = item % P2, g = item / P2;
#pragma unroll
        for (int t = 0; t < TT; ++t) {
            const int64_t pid = pbase + g * TT + t;
            if (pid >= npar) continue;
            int64_t tp, tr;
            target_of(pid, k, n, G, S, tp, tr);
            Lout[tr * S + r] = acc[it][t];
        }
    }
}

hipError_t launch_m2l_rot(int P, int L, void *const *B, void *const *Lc, const double *rot,
                          const double *tz, const int2 *cls, hipStream_t st) {
    if (L < 2) return hipSuccess;
    RotPlan pl{};
    pl.nlev = L - 1;
    int64_t nb = 0;
    for (int i = 0; i < pl.nlev; ++i) {
        const int l = L - i;
        const int64_t h = (int64_t)1 << (l - 1);
        pl.level[i] = l;
        pl.blk0[i] = nb;
        pl.B[i] = (const double *)B[l];
        pl.L[i] = (double *)Lc[l];
        nb += 8 * ((h * h * h + kRotNT - 1) / kRotNT);
    }
    pl.blk0[pl.nlev] = nb;
    switch (P) {
#define CASE(PP) \
    case PP: k_m2l_rot<PP><<<(unsigned)nb, kRotThreads, 0, st>>>(pl, rot, tz, cls); break;
        CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9)
        CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ host side
static int64_t level_tiles(int l) {
    const int64_t h = (int64_t)1 << (l - 1);
    return 8 * ((h * h * h + kTile - 1) / kTile);
}

// Plan: levels largest first.  Levels with at least one tile per CU run
// unsplit; the others share one split factor s, chosen by simulating the
// in-order dispatch of blocks onto ncu one-block-per-CU slots (a whole tile
// takes time 1, a part 1/s plus a small fixed overhead).
static M2LPlan compute_plan(int P, int L, bool allow_split, int ncu) {
    M2LPlan pl{};
    pl.nlev = L - 1;
    const int S = coef_stride(P);
    const int nch = (kOffsetsPerClass * (S / 8) + 3) / 4;  // K-steps of a tile
    int64_t big = 0, small = 0;
    for (int i = 0; i < pl.nlev; ++i) {
        const int l = L - i;
        pl.level[i] = l;
        pl.ntile[i] = level_tiles(l);
        if (pl.ntile[i] >= ncu) big += pl.ntile[i];
        else small += pl.ntile[i];
    }
    int best_s = 1;
    if (allow_split && small > 0 && ncu > 0) {
        const double ovh = 8.0 / nch;
        double best_t = 1e300;
        const int smax = std::max(1, std::min(8, nch / 32));
        for (int s = 1; s <= smax; ++s) {
            std::priority_queue<double, std::vector<double>, std::greater<double>> slots;
            for (int c = 0; c < ncu; ++c) slots.push(0.0);
            auto run = [&](int64_t cnt, double dur) {
                for (int64_t j = 0; j < cnt; ++j) {
                    const double t0 = slots.top();
                    slots.pop();
                    slots.push(t0 + dur);
                }
            };
            run(big, 1.0 + ovh);
            run(small * s, 1.0 / s + ovh);
            double t = 0;
            while (!slots.empty()) {
                t = slots.top();
                slots.pop();
            }
            if (t < best_t - 1e-9) {
                best_t = t;
                best_s = s;
            }
        }
    }
    int64_t nu = 0, np = 0, nf = 0;
    for (int i = 0; i < pl.nlev; ++i) {
        pl.nsplit[i] = pl.ntile[i] >= ncu ? 1 : best_s;
        pl.unit0[i] = nu;
        nu += pl.ntile[i] * pl.nsplit[i];
        pl.part0[i] = np;
        pl.fix0[i] = nf;
        if (pl.nsplit[i] > 1) {
            np += pl.ntile[i] * pl.nsplit[i];
            nf += pl.ntile[i];
        }
    }
    pl.unit0[pl.nlev] = nu;
    pl.fix0[pl.nlev] = nf;
    return pl;
}

// The plan depends only on (p, L, split allowed, CU count); the dispatch
// simulation costs tens of microseconds of host time, so plans are memoised.
static M2LPlan make_plan(int P, int L, bool allow_split, int ncu) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, bool, int>, M2LPlan> memo;
    const auto key = std::make_tuple(P, L, allow_split, ncu);
    std::lock_guard<std::mutex> g(mu);
    auto it = memo.find(key);
    if (it == memo.end()) it = memo.emplace(key, compute_plan(P, L, allow_split, ncu)).first;
    return it->second;
}

size_t m2l_partial_bytes(int P, int L, bool f64, int ncu) {
    (void)f64;  // both forms split the small levels and keep FP64 partial sums
    if (L < 2) return 0;
    const M2LPlan pl = make_plan(P, L, true, ncu);
    int64_t np = 0;
    for (int i = 0; i < pl.nlev; ++i)
        if (pl.nsplit[i] > 1) np += pl.ntile[i] * pl.nsplit[i];
    return (size_t)np * kTile * P * P * sizeof(double);
}

// Eight waves (two per SIMD) wherever their operator ring fits in LDS; four
// (one per SIMD) otherwise, i.e. for the 3-part split at p = 13.
template <int NSPLIT, int P, bool H = false>
static void launch_bf16(unsigned nb, const M2LPlan &pl, const uint16_t *A, size_t astride,
                        const int2 *cls, double *partial, hipStream_t st) {
    constexpr bool fits8 = MixCfg<NSPLIT, P, 8>::NA * MixCfg<NSPLIT, P, 8>::STAGE <= 150;
    if constexpr (fits8)
        k_m2l_bf16<NSPLIT, P, 8, H><<<nb, 512, 0, st>>>(pl, A, astride, cls, partial);
    else
        k_m2l_bf16<NSPLIT, P, 4, H><<<nb, 256, 0, st>>>(pl, A, astride, cls, partial);
}

// sum the K parts of the split tiles (after either form's kernel)
static hipError_t fixup(int P, const M2LPlan &pl, unsigned nfix, const double *partial, hipStream_t st) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nfix == 0) return e;
    const int64_t total = (int64_t)nfix * kTile * P * P;
    k_m2l_fixup<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(P, pl, partial, total);
    return hipGetLastError();
}

hipError_t launch_m2l(int P, int L, bool f64, int nsplit, void *const *B, void *const *Lc,
                      const int *out_f64, const void *A, size_t astride, const int2 *cls,
                      double *partial, size_t partial_bytes, int ncu, const M2LHalf *half,
                      hipStream_t st) {
    if (L < 2) return hipSuccess;
    M2LPlan pl = make_plan(P, L, true, ncu);
    pl.lmax = half ? half->lmax : nullptr;
    pl.oscale = half ? half->oscale : nullptr;
    for (int i = 0; i < pl.nlev; ++i) {
        const int l = pl.level[i];
        pl.B[i] = B[l];
        pl.L[i] = Lc[l];
        pl.out_f64[i] = out_f64[l];
    }
    const unsigned nb = (unsigned)pl.unit0[pl.nlev];
    const unsigned nfix = (unsigned)pl.fix0[pl.nlev];
    if (nfix > 0 && (!partial || partial_bytes < m2l_partial_bytes(P, L, f64, ncu)))
        return hipErrorInvalidValue;
    if (f64) {
        switch (P) {
#define CASE(PP) \
    case PP: k_m2l_f64<PP><<<nb, 256, 0, st>>>(pl, (const double *)A, cls, partial); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
            CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
            default: return hipErrorInvalidValue;
        }
        return fixup(P, pl, nfix, partial, st);
    }
    if (half) {
        if (!half->lmax || !half->oscale) return hipErrorInvalidValue;
        switch (P) {
#define CASEH(PP) \
    case PP: launch_bf16<2, PP, true>(nb, pl, (const uint16_t *)A, astride, cls, partial, st); break;
            CASEH(1) CASEH(2) CASEH(3) CASEH(4) CASEH(5) CASEH(6) CASEH(7) CASEH(8)
            CASEH(9) CASEH(10) CASEH(11) CASEH(12) CASEH(13) CASEH(14) CASEH(15) CASEH(16)
#undef CASEH
            default: return hipErrorInvalidValue;
        }
        return fixup(P, pl, nfix, partial, st);
    }
    if (nsplit == 3 && P > kMixedSplit3PMax) return hipErrorInvalidValue;
#define CASE3(PP) \
    case PP: launch_bf16<3, PP>(nb, pl, (const uint16_t *)A, astride, cls, partial, st); break;
#define CASE2(PP) \
    case PP: launch_bf16<2, PP>(nb, pl, (const uint16_t *)A, astride, cls, partial, st); break;
    if (nsplit == 3) {
        switch (P) {
            CASE3(1) CASE3(2) CASE3(3) CASE3(4) CASE3(5) CASE3(6) CASE3(7) CASE3(8)
            CASE3(9) CASE3(10) CASE3(11) CASE3(12) CASE3(13)
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (P) {
            CASE2(1) CASE2(2) CASE2(3) CASE2(4) CASE2(5) CASE2(6) CASE2(7) CASE2(8)
            CASE2(9) CASE2(10) CASE2(11) CASE2(12) CASE2(13) CASE2(14) CASE2(15) CASE2(16)
            default: return hipErrorInvalidValue;
        }
    }
#undef CASE3
#undef CASE2
    return fixup(P, pl, nfix, partial, st);
}

}  // namespace fmm

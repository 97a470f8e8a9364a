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
// Mixed form: operands split into bf16 parts x = x0 + x1 (+ x2); the products
// x_i y_j with i + j < parts are accumulated by v_mfma_f32_16x16x32_bf16 in
// FP32 and merged into FP64 accumulators every 8 K-chunks (256 terms).
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

template <int NSPLIT, int RT, int NB>
__global__ __launch_bounds__(256) void k_m2l_bf16(int P, int l, const uint16_t *__restrict__ B,
                                                  size_t bstride, const uint16_t *__restrict__ A,
                                                  size_t astride, const int2 *__restrict__ cls,
                                                  void *__restrict__ Lout, int out_f64) {
    const int S = coef_stride(P), PPO = S / 8, P2 = P * P, R = RT * 16;
    const int n = 1 << l, h = n >> 1;
    const int64_t G = n + 6;
    const int k = blockIdx.y;
    const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int64_t npar = (int64_t)h * h * h;

    int64_t tpad[NB], trow[NB];
    bool cvalid[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int64_t pid = ((int64_t)blockIdx.x * 4 + wave) * NB * 16 + b * 16 + col;
        cvalid[b] = pid < npar;
        const int64_t pc = cvalid[b] ? pid : 0;
        const int64_t tx = 2 * (pc % h) + kx, ty = 2 * ((pc / h) % h) + ky,
                      tz = 2 * (pc / ((int64_t)h * h)) + kz;
        tpad[b] = (tx + 3) + G * ((ty + 3) + G * (tz + 3));
        trow[b] = tx + (int64_t)n * (ty + (int64_t)n * tz);
    }

    f32x4 acc[RT][NB];
    f64x4 acc64[RT][NB];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            acc[r][b] = f32x4{0, 0, 0, 0};
            acc64[r][b] = f64x4{0, 0, 0, 0};
        }

    const int NPC = kOffsetsPerClass * PPO;
    const int NCH = (NPC + 3) / 4;
    const int2 *ctab = cls + k * kOffsetsPerClass;
    for (int kc = 0; kc < NCH; ++kc) {
        const int g = 4 * kc + q;
        bf16x8 bfr[NSPLIT][NB], afr[NSPLIT][RT];
        if (g < NPC) {
            const int slot = g / PPO, cp = g - slot * PPO;
            const int2 e = ctab[slot];
            const int64_t delta = unpack_delta(e.x, G);
#pragma unroll
            for (int s = 0; s < NSPLIT; ++s) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    bfr[s][b] = *(const bf16x8 *)(B + s * bstride + (size_t)(tpad[b] + delta) * S + 8 * cp);
#pragma unroll
                for (int r = 0; r < RT; ++r)
                    afr[s][r] = *(const bf16x8 *)(A + s * astride +
                                                  ((size_t)e.y * R + 16 * r + col) * S + 8 * cp);
            }
        } else {
#pragma unroll
            for (int s = 0; s < NSPLIT; ++s) {
#pragma unroll
                for (int b = 0; b < NB; ++b) bfr[s][b] = bf16x8{};
#pragma unroll
                for (int r = 0; r < RT; ++r) afr[s][r] = bf16x8{};
            }
        }
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < NSPLIT; ++i)
#pragma unroll
                    for (int j = 0; i + j < NSPLIT; ++j)
                        acc[r][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[i][r], bfr[j][b],
                                                                           acc[r][b], 0, 0, 0);
        if ((kc & 7) == 7 || kc == NCH - 1) {
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc64[r][b][i] += (double)acc[r][b][i];
                    acc[r][b] = f32x4{0, 0, 0, 0};
                }
        }
    }
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
}

template <int RT, int NB>
__global__ __launch_bounds__(256) void k_m2l_f64(int P, int l, const double *__restrict__ B,
                                                 const double *__restrict__ A,
                                                 const int2 *__restrict__ cls,
                                                 double *__restrict__ Lout) {
    const int S = coef_stride(P), P2 = P * P, R = RT * 16;
    const int n = 1 << l, h = n >> 1;
    const int64_t G = n + 6;
    const int k = blockIdx.y;
    const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int64_t npar = (int64_t)h * h * h;

    int64_t tpad[NB], trow[NB];
    bool cvalid[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int64_t pid = ((int64_t)blockIdx.x * 4 + wave) * NB * 16 + b * 16 + col;
        cvalid[b] = pid < npar;
        const int64_t pc = cvalid[b] ? pid : 0;
        const int64_t tx = 2 * (pc % h) + kx, ty = 2 * ((pc / h) % h) + ky,
                      tz = 2 * (pc / ((int64_t)h * h)) + kz;
        tpad[b] = (tx + 3) + G * ((ty + 3) + G * (tz + 3));
        trow[b] = tx + (int64_t)n * (ty + (int64_t)n * tz);
    }
    f64x4 acc[RT][NB];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[r][b] = f64x4{0, 0, 0, 0};

    const int NK = kOffsetsPerClass * P2;
    const int NCH = (NK + 3) / 4;
    const int2 *ctab = cls + k * kOffsetsPerClass;
    for (int kc = 0; kc < NCH; ++kc) {
        const int g = 4 * kc + q;
        double bv[NB], av[RT];
        if (g < NK) {
            const int slot = g / P2, c = g - slot * P2;
            const int2 e = ctab[slot];
            const int64_t delta = unpack_delta(e.x, G);
#pragma unroll
            for (int b = 0; b < NB; ++b) bv[b] = B[(size_t)(tpad[b] + delta) * S + c];
#pragma unroll
            for (int r = 0; r < RT; ++r) av[r] = A[((size_t)e.y * R + 16 * r + col) * S + c];
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b) bv[b] = 0.0;
#pragma unroll
            for (int r = 0; r < RT; ++r) av[r] = 0.0;
        }
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int b = 0; b < NB; ++b)
                acc[r][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r], bv[b], acc[r][b], 0, 0, 0);
    }
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

template <int NSPLIT, int RT>
static void go_bf16(int P, int l, const uint16_t *B, size_t bs, const uint16_t *A, size_t as,
                    const int2 *cls, void *Lout, int out_f64, hipStream_t st) {
    constexpr int NB = RT <= 8 ? 2 : 1;
    const int64_t h = (int64_t)1 << (l - 1);
    const int64_t npar = h * h * h;
    const dim3 grid((unsigned)((npar + 4 * NB * 16 - 1) / (4 * NB * 16)), 8);
    k_m2l_bf16<NSPLIT, RT, NB><<<grid, 256, 0, st>>>(P, l, B, bs, A, as, cls, Lout, out_f64);
}

template <int RT>
static void go_f64(int P, int l, const double *B, const double *A, const int2 *cls, double *Lout,
                   hipStream_t st) {
    constexpr int NB = RT <= 8 ? 2 : 1;
    const int64_t h = (int64_t)1 << (l - 1);
    const int64_t npar = h * h * h;
    const dim3 grid((unsigned)((npar + 4 * NB * 16 - 1) / (4 * NB * 16)), 8);
    k_m2l_f64<RT, NB><<<grid, 256, 0, st>>>(P, l, B, A, cls, Lout);
}

hipError_t launch_m2l_bf16(int P, int l, int nsplit, const uint16_t *B, size_t bstride,
                           const uint16_t *A, size_t astride, const int2 *cls, void *Lout,
                           int out_f64, hipStream_t st) {
    const int RT = m2l_rows(P) / 16;
#define CASE(RR)                                                                        \
    case RR:                                                                            \
        if (nsplit == 3)                                                                \
            go_bf16<3, RR>(P, l, B, bstride, A, astride, cls, Lout, out_f64, st);       \
        else                                                                            \
            go_bf16<2, RR>(P, l, B, bstride, A, astride, cls, Lout, out_f64, st);       \
        break;
    switch (RT) {
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
        default: return hipErrorInvalidValue;
    }
#undef CASE
    return hipGetLastError();
}

hipError_t launch_m2l_f64(int P, int l, const double *B, const double *A, const int2 *cls,
                          double *Lout, hipStream_t st) {
    const int RT = m2l_rows(P) / 16;
#define CASE(RR) \
    case RR: go_f64<RR>(P, l, B, A, cls, Lout, st); break;
    switch (RT) {
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
        default: return hipErrorInvalidValue;
    }
#undef CASE
    return hipGetLastError();
}

}  // namespace fmm

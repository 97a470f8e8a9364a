// tree.hip -- uniform octree build on the GPU: Morton keys, leaf histogram,
// level selection counters, exclusive scan, stable counting sort and the
// gather of leaf-relative coordinates (Sec. 2.1 subdivision; Sec. 5 index
// sorting with start/offset access and Morton-indexed uniform trees).
#include "kernels.hpp"

namespace fmm {

// Box coordinate at level 10 of one coordinate value: floor(s * 1024) clamped
// to [0, 1023] with s = (x - lo) / size in FP64.  The coordinate at level l is
// this value >> (10 - l), which equals min(floor(s * 2^l), 2^l - 1).
__device__ inline uint32_t box10(double x, double lo, double size) {
    const double s = (x - lo) / size;
    double v = floor(s * 1024.0);
    v = v > 1023.0 ? 1023.0 : v;
    v = v < 0.0 ? 0.0 : v;
    return (uint32_t)v;
}

// Zero the leaf counters of a level (nb words) and nctr build counters.
__global__ void k_zero(int64_t nb, uint32_t *__restrict__ cnt, unsigned int *__restrict__ ctr,
                       int nctr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) cnt[i] = 0;
    if (i < nctr) ctr[i] = 0;
}

// Key of every particle, and its leaf count at the level of `shift`: the
// value returned by the count's atomic add is the particle's rank within its
// leaf (arrival order; the leaf is put in input order afterwards by k_fixup).
// A position outside the root cube or not finite is counted in nbad and
// given key 0, so that the rest of the build stays in bounds.
template <typename T>
__global__ void k_keys(int64_t n, const T *__restrict__ pos, double lo0, double lo1, double lo2,
                       double size, int shift, uint32_t *__restrict__ key10,
                       uint32_t *__restrict__ cnt, uint32_t *__restrict__ rank,
                       unsigned int *__restrict__ nbad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = (double)pos[3 * i], y = (double)pos[3 * i + 1], z = (double)pos[3 * i + 2];
    const bool ok = (x >= lo0 && x <= lo0 + size) && (y >= lo1 && y <= lo1 + size) &&
                    (z >= lo2 && z <= lo2 + size);  // false for NaN
    uint32_t k = 0;
    if (ok)
        k = morton3(box10(x, lo0, size), box10(y, lo1, size), box10(z, lo2, size));
    else
        atomicAdd(nbad, 1u);
    key10[i] = k;
    if (cnt) rank[i] = atomicAdd(&cnt[k >> shift], 1u);
}

// Leaf counts and ranks at another level, from the keys.
__global__ void k_hist(int64_t n, const uint32_t *__restrict__ key10, int shift,
                       uint32_t *__restrict__ cnt, uint32_t *__restrict__ rank) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    rank[i] = atomicAdd(&cnt[key10[i] >> shift], 1u);
}

__global__ void k_max(int64_t nb, const uint32_t *__restrict__ cnt, unsigned int *__restrict__ mx) {
    __shared__ unsigned int red[256];
    unsigned int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, cnt[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomic_max_shared(mx, red[0]);
}

// Exclusive scan in blocks of 4096 (1024 threads x 4); block totals to sums.
__global__ __launch_bounds__(1024) void k_scan_blocks(int64_t nb, const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out,
                                                      uint32_t *__restrict__ sums) {
    __shared__ uint32_t ws[16];
    const int64_t base = (int64_t)blockIdx.x * 4096 + 4 * threadIdx.x;
    uint32_t v[4], t = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < nb) ? in[base + k] : 0u;
        t += v[k];
    }
    // inclusive scan of t across the block: wave scan then wave totals
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = t;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();
    if (threadIdx.x < 16) {
        uint32_t s = ws[threadIdx.x];
        for (int d = 1; d < 16; d <<= 1) {
            const uint32_t y = __shfl_up(s, d, 16);
            if ((int)threadIdx.x >= d) s += y;
        }
        ws[threadIdx.x] = s;
    }
    __syncthreads();
    uint32_t excl = x - t + (wave > 0 ? ws[wave - 1] : 0u);
    for (int k = 0; k < 4; ++k) {
        if (base + k < nb) out[base + k] = excl;
        excl += v[k];
    }
    if (threadIdx.x == 1023 && sums) sums[blockIdx.x] = excl;
}

// Exclusive scan and maximum of up to kScan1 counts in one block, staged in
// LDS: coalesced load, thread t scans counts 32 t .. 32 t + 31 (LDS word
// i + i / 32, so the 32-word stride hits distinct banks), coalesced store;
// out[nb] receives the total, *mx the maximum.
constexpr int64_t kScan1 = 32768;

__device__ __forceinline__ int scan1_slot(int i) { return i + (i >> 5); }

__global__ __launch_bounds__(1024) void k_scan_max1(int64_t nb, const uint32_t *__restrict__ in,
                                                    uint32_t *__restrict__ out,
                                                    unsigned int *__restrict__ mx,
                                                    const unsigned int *__restrict__ nbad,
                                                    unsigned int *host) {
    __shared__ uint32_t buf[kScan1 + kScan1 / 32];
    __shared__ uint32_t ws[16], wm[16];
    const int n = (int)nb, tid = threadIdx.x;
    uint32_t v[32], t = 0, m = 0;
#pragma unroll
    for (int k = 0; k < 32; ++k) {  // all 32 loads in flight at once
        const int i = tid + 1024 * k;
        v[k] = i < n ? in[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) buf[scan1_slot(tid + 1024 * k)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        v[k] = buf[scan1_slot(32 * tid + k)];
        t += v[k];
        m = max(m, v[k]);
    }
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t x = t;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
        m = max(m, (uint32_t)__shfl_xor(m, d, 64));
    }
    if (lane == 63) ws[wave] = x;
    if (lane == 0) wm[wave] = m;
    __syncthreads();
    if (tid < 16) {
        uint32_t s = ws[tid], mm = wm[tid];
        for (int d = 1; d < 16; d <<= 1) {
            const uint32_t y = __shfl_up(s, d, 16);
            if (tid >= d) s += y;
            mm = max(mm, (uint32_t)__shfl_xor(mm, d, 16));
        }
        ws[tid] = s;
        if (tid == 0) {
            *mx = mm;
            // the two build counters straight into the caller's pinned host
            // words (no copy on the stream): positions out of the domain
            // (final since the key pass ended) and the fullest leaf
            if (host) {
                host[0] = *nbad;
                host[1] = mm;
                __threadfence_system();
            }
        }
    }
    __syncthreads();
    uint32_t excl = x - t + (wave > 0 ? ws[wave - 1] : 0u);
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        buf[scan1_slot(32 * tid + k)] = excl;
        excl += v[k];
    }
    if (tid == 1023) out[n] = excl;
    __syncthreads();
    for (int i = tid; i < n; i += 1024) out[i] = buf[scan1_slot(i)];
}

// adds the scanned block sums; also writes the total (sums[nblocks]) to out[nb]
__global__ void k_scan_add(int64_t nb, int64_t nblocks, uint32_t *__restrict__ out,
                           const uint32_t *__restrict__ sums) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) out[nb] = sums[nblocks];
    if (i >= nb) return;
    out[i] += sums[i / 4096];
}

// Counting sort placement: leaf start + rank within the leaf (no atomics).
__global__ void k_place(int64_t n, const uint32_t *__restrict__ key10, int shift,
                        const uint32_t *__restrict__ rank, const uint32_t *__restrict__ start,
                        uint32_t *__restrict__ tmp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tmp[start[key10[i] >> shift] + rank[i]] = (uint32_t)i;
}

// One wave per leaf (four leaves per 256-thread block): orders the leaf's
// particles by input index (making the counting sort stable and the whole
// build deterministic), writes perm and the particles' coordinates relative
// to the leaf centre in units of the leaf width, u = s 2^L - (i + 1/2) in
// [-1/2, 1/2], computed in FP64 and stored as FP64 (plain form) or rounded to
// 32-bit fixed point (mixed form).  A leaf of more than kFixupCache particles
// (possible only at the deepest level) ranks from global memory.
constexpr int kFixupCache = 512;
constexpr int64_t kFixupBlocks = 16384;

// A leaf of more than `skip` particles is left as it is: the host sorts at
// a finer level when a leaf is over the cap below the deepest level, so the
// quadratic ranking of such a leaf would be wasted.
template <typename T>
__global__ __launch_bounds__(256) void k_fixup(int L, uint32_t skip, const uint32_t *__restrict__ start,
                                               const uint32_t *__restrict__ tmp,
                                               const T *__restrict__ pos, double lo0, double lo1,
                                               double lo2, double size, uint32_t *__restrict__ perm,
                                               int4 *__restrict__ xyz32, double4 *__restrict__ xyz64) {
    __shared__ uint32_t idxs[4][kFixupCache];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t nleaf = 1u << (3 * L);
    uint32_t *const idx = idxs[wave];
    const double scale = (double)(1u << L);
    // Wave w of the W in the grid takes the leaves w, w + W, w + 2W, ... (no
    // block barrier), 64 at a time: the lanes read 64 counts at once and the
    // wave then works through the leaves that need it.  A tree of mostly
    // empty bins costs one load per 64 of them, and a wave's leaves lie far
    // apart, so that a dense region of the input is spread over many waves.
    const uint32_t W = 4 * gridDim.x, w = 4 * blockIdx.x + wave;
    for (uint32_t base = w; base < nleaf; base += 64 * W) {
        const uint32_t mine = base + lane * W;
        const uint32_t c_l = mine < nleaf ? start[mine + 1] - start[mine] : 0;
        uint64_t todo = __ballot(c_l != 0 && c_l <= skip);
        while (todo) {
            const int b = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t leaf = base + (uint32_t)b * W;
            const uint32_t s0 = start[leaf], cnt = start[leaf + 1] - s0;
            const bool cached = cnt <= (uint32_t)kFixupCache;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // the previous leaf's reads of idx
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (cached)
                for (uint32_t j = lane; j < cnt; j += 64) idx[j] = tmp[s0 + j];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double bx = (double)compact3(leaf) + 0.5, by = (double)compact3(leaf >> 1) + 0.5,
                         bz = (double)compact3(leaf >> 2) + 0.5;
            for (uint32_t j = lane; j < cnt; j += 64) {
                const uint32_t me = cached ? idx[j] : tmp[s0 + j];
                uint32_t rank = 0;
                if (cached) {
                    for (uint32_t k = 0; k < cnt; ++k) rank += idx[k] < me;
                } else {
                    for (uint32_t k = 0; k < cnt; ++k) rank += tmp[s0 + k] < me;
                }
                const uint32_t d = s0 + rank;
                perm[d] = me;
                const double ux = ((double)pos[3 * (size_t)me] - lo0) / size * scale - bx;
                const double uy = ((double)pos[3 * (size_t)me + 1] - lo1) / size * scale - by;
                const double uz = ((double)pos[3 * (size_t)me + 2] - lo2) / size * scale - bz;
                if (xyz32) {
                    // fixed point in [-2^29, 2^29 - 1]: u = +1/2 (a point on the upper
                    // face of the root cube) moves by 2^-30 leaf widths
                    const int top = (1 << 29) - 1;
                    xyz32[d] = make_int4(min(__double2int_rn(ux * kFixScale), top),
                                         min(__double2int_rn(uy * kFixScale), top),
                                         min(__double2int_rn(uz * kFixScale), top), 0);
                }
                if (xyz64) xyz64[d] = make_double4(ux, uy, uz, 0.0);
            }
        }
    }
}

// ----------------------------------------------------- key sort (adaptive)
// Stable LSD radix sort of the particles by their key at a level (the 3L
// high bits of the level-10 key), 8 bits a pass, for trees whose finest
// level is too deep for a bin per key (8^L bins): the first pass takes the
// input order as the values, so ties keep input order and the last pass's
// values are the permutation (sorted position -> input index); the last
// pass also writes the sorted keys.  A block takes 4096 elements, element
// j * 256 + t of its range in thread t's step j (so the steps in order visit
// the block's elements in index order).  Per pass one kernel writes each
// block's digit histogram, digit-major (a scan then gives every (digit,
// block) its output offset), and one places each element at its offset plus
// its rank among the block's earlier elements of the same digit: within a
// wave from ballots on the digit's bits, across waves and steps from LDS
// counts.
constexpr int kKsSteps = 16, kKsBlock = 256 * kKsSteps;

__device__ __forceinline__ uint32_t ks_key(bool first, int64_t e, const uint32_t *__restrict__ key10, int shift,
                                           const uint32_t *__restrict__ kin) {
    return first ? key10[e] >> shift : kin[e];
}

__global__ __launch_bounds__(256) void k_ks_hist(int64_t n, int64_t nblocks, int first,
                                                 const uint32_t *__restrict__ key10, int shift,
                                                 const uint32_t *__restrict__ kin, int bit, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kKsBlock;
    for (int j = 0; j < kKsSteps; ++j) {
        const int64_t e = base + j * 256 + threadIdx.x;
        if (e < n) atomicAdd(&h[(ks_key(first, e, key10, shift, kin) >> bit) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_ks_scatter(int64_t n, int64_t nblocks, int first,
                                                    const uint32_t *__restrict__ key10, int shift,
                                                    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                    int bit, const uint32_t *__restrict__ off,
                                                    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout) {
    __shared__ uint32_t wcnt[2][4][256];  // per step parity and wave: the step's count of each digit
    __shared__ uint32_t run[256];         // the block's elements of each digit in earlier steps
    __shared__ uint32_t goff[256];        // the block's output offset of each digit
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    goff[tid] = off[(int64_t)tid * nblocks + blockIdx.x];
    run[tid] = 0;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * kKsBlock;
    for (int j = 0; j < kKsSteps; ++j) {
        const int64_t e = base + j * 256 + tid;
        const bool valid = e < n;
        const uint32_t key = valid ? ks_key(first, e, key10, shift, kin) : 0u;
        const uint32_t d = (key >> bit) & 255u;
        // this wave's row of counts of this step's parity, cleared: it was
        // last read two steps back, before the previous step's first barrier
        uint32_t(*const cnt)[256] = wcnt[j & 1];
#pragma unroll
        for (int i = 0; i < 4; ++i) cnt[wave][lane + 64 * i] = 0u;
        // the lanes of the wave holding the same digit
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint64_t bk = __ballot(valid && ((d >> k) & 1u));
            m &= ((d >> k) & 1u) ? bk : ~bk;
        }
        __syncthreads();  // the rows are cleared
        if (valid && (m & below) == 0) cnt[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t r = run[d] + (uint32_t)__popcll(m & below);
            for (int w = 0; w < wave; ++w) r += cnt[w][d];
            const uint32_t dst = goff[d] + r;
            kout[dst] = key;
            vout[dst] = first ? (uint32_t)e : vin[e];
        }
        __syncthreads();  // every read of run of this step is done
        run[tid] += cnt[0][tid] + cnt[1][tid] + cnt[2][tid] + cnt[3][tid];
    }
}

__global__ void k_iota(int64_t n, uint32_t *__restrict__ v, uint32_t *__restrict__ zero) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        v[i] = (uint32_t)i;
        zero[i] = 0u;
    }
}

// Sorted records: for sorted position d the particle perm[d] relative to its
// leaf centre in units of the leaf width, u = s 2^L - (i + 1/2), computed in
// FP64 as the fix-up does.
template <typename T>
__global__ void k_records(int64_t n, int L, const uint32_t *__restrict__ perm, const uint32_t *__restrict__ key10,
                          const T *__restrict__ pos, double lo0, double lo1, double lo2, double size,
                          double4 *__restrict__ xyz64) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const uint32_t me = perm[d];
    const uint32_t leaf = key10[me] >> (3 * (10 - L));
    const double scale = (double)(1u << L);
    const double bx = (double)compact3(leaf) + 0.5, by = (double)compact3(leaf >> 1) + 0.5,
                 bz = (double)compact3(leaf >> 2) + 0.5;
    const double ux = ((double)pos[3 * (size_t)me] - lo0) / size * scale - bx;
    const double uy = ((double)pos[3 * (size_t)me + 1] - lo1) / size * scale - by;
    const double uz = ((double)pos[3 * (size_t)me + 2] - lo2) / size * scale - bz;
    xyz64[d] = make_double4(ux, uy, uz, 0.0);
}

// First sorted position of every key at level cl (cstart[x], x in
// [0, 8^cl]) from the keys at level L >= cl sorted: a binary search per x
// (an empty stretch of keys costs no thread more than another).
__global__ void k_key_starts(int64_t n, int sh, const uint32_t *__restrict__ skey, int64_t nc,
                             uint32_t *__restrict__ cstart) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > nc) return;
    int64_t lo = 0, hi = n;  // first d with skey[d] >> sh >= x
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)(skey[mid] >> sh) < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    cstart[x] = (uint32_t)lo;
}

// Per leaf: n_t * (sum of counts over the near leaves) ; summed in int64.
__global__ void k_pair_count(int L, const uint32_t *__restrict__ start,
                             unsigned long long *__restrict__ out) {
    const uint32_t nleaf = 1u << (3 * L);
    const uint32_t leaf = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = 0;
    if (leaf < nleaf) {
        const int side = 1 << L;
        const int ix = compact3(leaf), iy = compact3(leaf >> 1), iz = compact3(leaf >> 2);
        const unsigned long long nt = start[leaf + 1] - start[leaf];
        unsigned long long ns = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int x = ix + dx, y = iy + dy, z = iz + dz;
                    if (x < 0 || y < 0 || z < 0 || x >= side || y >= side || z >= side) continue;
                    const uint32_t s = morton3(x, y, z);
                    ns += start[s + 1] - start[s];
                }
        v = nt * ns;
    }
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}

// ------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_keys(int64_t n, int dtype, const void *pos, const double lo[3], double size,
                       int level, uint32_t *key10, uint32_t *cnt, uint32_t *rank,
                       unsigned int *counters, hipStream_t st) {
    // without cnt, the keys alone (for the key sort)
    const int64_t nb = cnt ? (int64_t)1 << (3 * level) : 0;
    // counters: [0] positions out of the domain, [1] largest leaf count
    k_zero<<<nblk(std::max<int64_t>(nb, 2), 256), 256, 0, st>>>(nb, cnt, counters, 2);
    const int shift = 3 * (10 - level);
    if (dtype == FMM_F64)
        k_keys<double><<<nblk(n, 256), 256, 0, st>>>(n, (const double *)pos, lo[0], lo[1], lo[2],
                                                      size, shift, key10, cnt, rank, counters);
    else
        k_keys<float><<<nblk(n, 256), 256, 0, st>>>(n, (const float *)pos, lo[0], lo[1], lo[2],
                                                     size, shift, key10, cnt, rank, counters);
    return hipGetLastError();
}

hipError_t launch_zero(uint32_t *p, int64_t words, hipStream_t st) {
    if (words <= 0) return hipSuccess;
    k_zero<<<nblk(words, 256), 256, 0, st>>>(words, p, nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_hist(int64_t n, const uint32_t *key10, int level, uint32_t *cnt, uint32_t *rank,
                       unsigned int *counters, hipStream_t st) {
    const int64_t nb = (int64_t)1 << (3 * level);
    // counters[1] (the largest leaf count) restarts; counters[0] keeps its value
    k_zero<<<nblk(nb, 256), 256, 0, st>>>(nb, cnt, counters + 1, 1);
    k_hist<<<nblk(n, 256), 256, 0, st>>>(n, key10, 3 * (10 - level), cnt, rank);
    return hipGetLastError();
}

// scratch must hold scan_scratch_words(nb) words: per recursion level the
// block sums and their scan (with total), then the next level's scratch
int64_t scan_scratch_words(int64_t nb) {
    const int64_t nblocks = (nb + 4095) / 4096;
    if (nblocks <= 1) return 1;
    return 2 * nblocks + 1 + scan_scratch_words(nblocks);
}

hipError_t launch_scan(int64_t nb, const uint32_t *in, uint32_t *out, uint32_t *scratch,
                       hipStream_t st) {
    // out[0..nb) exclusive scan, out[nb] total.  Recursive over block sums.
    const int64_t nblocks = (nb + 4095) / 4096;
    if (nblocks == 1) {
        k_scan_blocks<<<1, 1024, 0, st>>>(nb, in, out, out + nb);
        return hipGetLastError();
    }
    uint32_t *sums = scratch;
    uint32_t *sums_scan = scratch + nblocks;
    k_scan_blocks<<<(unsigned)nblocks, 1024, 0, st>>>(nb, in, out, sums);
    hipError_t e = launch_scan(nblocks, sums, sums_scan, sums_scan + nblocks + 1, st);
    if (e != hipSuccess) return e;
    k_scan_add<<<nblk(nb, 256), 256, 0, st>>>(nb, nblocks, out, sums_scan);
    return hipGetLastError();
}

hipError_t launch_scan_max(int64_t nb, const uint32_t *in, uint32_t *out, uint32_t *scratch,
                           unsigned int *mx, const unsigned int *nbad, unsigned int *host, bool *host_done,
                           hipStream_t st) {
    if (host_done) *host_done = false;
    if (nb <= kScan1) {
        k_scan_max1<<<1, 1024, 0, st>>>(nb, in, out, mx, nbad, host);
        if (host_done) *host_done = host != nullptr;
        return hipGetLastError();
    }
    // larger trees: the maximum (into *mx, zeroed by the key or histogram
    // pass) and the multi-block scan
    k_max<<<(unsigned)std::min<int64_t>(1024, (nb + 255) / 256), 256, 0, st>>>(nb, in, mx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_scan(nb, in, out, scratch, st);
}

hipError_t launch_sort(int64_t n, int level, uint32_t skip, const uint32_t *key10, const uint32_t *rank,
                       const uint32_t *start, uint32_t *tmp, int dtype, const void *pos,
                       const double lo[3], double size, uint32_t *perm, int4 *xyz32,
                       double4 *xyz64, hipStream_t st) {
    const int64_t nb = (int64_t)1 << (3 * level);
    k_place<<<nblk(n, 256), 256, 0, st>>>(n, key10, 3 * (10 - level), rank, start, tmp);
    // four leaves per block, at most kFixupBlocks blocks striding over the rest
    const unsigned fix_blocks = (unsigned)std::min<int64_t>((nb + 3) / 4, kFixupBlocks);
    if (dtype == FMM_F64)
        k_fixup<double><<<fix_blocks, 256, 0, st>>>(level, skip, start, tmp, (const double *)pos, lo[0],
                                                       lo[1], lo[2], size, perm, xyz32, xyz64);
    else
        k_fixup<float><<<fix_blocks, 256, 0, st>>>(level, skip, start, tmp, (const float *)pos, lo[0],
                                                      lo[1], lo[2], size, perm, xyz32, xyz64);
    return hipGetLastError();
}

hipError_t launch_pair_count(int level, const uint32_t *start, unsigned long long *out,
                             hipStream_t st) {
    const int64_t nb = (int64_t)1 << (3 * level);
    hipError_t e = hipMemsetAsync(out, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    k_pair_count<<<nblk(nb, 256), 256, 0, st>>>(level, start, out);
    return hipGetLastError();
}

int64_t key_sort_hist_words(int64_t n) { return 256 * ((n + kKsBlock - 1) / kKsBlock); }

hipError_t launch_key_sort(int64_t n, int level, const uint32_t *key10, const KeySortWork &w, uint32_t *perm,
                           uint32_t *skey, hipStream_t st) {
    const int passes = (3 * level + 7) / 8, shift = 3 * (10 - level);
    const int64_t nblocks = (n + kKsBlock - 1) / kKsBlock;
    if (passes == 0) {
        k_iota<<<nblk(n, 256), 256, 0, st>>>(n, perm, skey);
        return hipGetLastError();
    }
    // values alternate between perm and w.vals so that the last pass writes
    // perm; keys between two buffers, the last pass writing skey
    const uint32_t *kin = nullptr, *vin = nullptr;
    for (int p = 0; p < passes; ++p) {
        const int back = passes - 1 - p;  // passes after this one
        uint32_t *kout = back == 0 ? skey : ((p & 1) ? w.keys_b : w.keys_a);
        uint32_t *vout = (back & 1) ? w.vals : perm;
        k_ks_hist<<<(unsigned)nblocks, 256, 0, st>>>(n, nblocks, p == 0, key10, shift, kin, 8 * p, w.hist);
        hipError_t e = launch_scan(256 * nblocks, w.hist, w.off, w.scan, st);
        if (e != hipSuccess) return e;
        k_ks_scatter<<<(unsigned)nblocks, 256, 0, st>>>(n, nblocks, p == 0, key10, shift, kin, vin, 8 * p, w.off,
                                                        kout, vout);
        kin = kout;
        vin = vout;
    }
    return hipGetLastError();
}

hipError_t launch_records(int64_t n, int level, const uint32_t *perm, const uint32_t *key10, int dtype,
                          const void *pos, const double lo[3], double size, double4 *xyz64, hipStream_t st) {
    if (dtype == FMM_F64)
        k_records<double><<<nblk(n, 256), 256, 0, st>>>(n, level, perm, key10, (const double *)pos, lo[0], lo[1],
                                                        lo[2], size, xyz64);
    else
        k_records<float><<<nblk(n, 256), 256, 0, st>>>(n, level, perm, key10, (const float *)pos, lo[0], lo[1],
                                                       lo[2], size, xyz64);
    return hipGetLastError();
}

hipError_t launch_key_starts(int64_t n, int level, int cl, const uint32_t *skey, uint32_t *cstart, hipStream_t st) {
    const int64_t nc = (int64_t)1 << (3 * cl);
    k_key_starts<<<nblk(nc + 1, 256), 256, 0, st>>>(n, 3 * (level - cl), skey, nc, cstart);
    return hipGetLastError();
}

}  // namespace fmm

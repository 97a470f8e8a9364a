// adaptive.hip -- the adaptive octree on the GPU (the adaptive construction
// that Sec. 5, future directions, names next to the uniform one).
//
// Tree.  Particles are counting-sorted by their Morton key at the finest
// level Lf (stable, ties in input order), so every box of every level is one
// contiguous range of the sorted order.  Level by level, a box holding more
// than leaf_max particles (below Lf) is split and its non-empty children are
// appended to the next level in Morton order; the rest are leaves.  Box ids
// are global (levels concatenated, breadth first), box 0 is the root.
//
// Lists, for box b (colleagues: the boxes of b's own level at offsets -1..1;
// two boxes are adjacent when their closed cubes touch and neither contains
// the other):
//   U(b), b a leaf: b and every leaf adjacent to b                    (P2P)
//   V(b): the children of the colleagues of b's parent not adjacent to b
//         (M2L; the 189 offsets of b's child class, absent sources empty)
//   W(b), b a leaf: descendants of b's colleagues not adjacent to b whose
//         parent is                                                   (M2P)
//   X(b): the leaves c with b in W(c)                                 (P2L)
// U, W and X are built by one thread per (box, colleague direction) walking
// the tree in a fixed order, so the lists, and the sums over them, are the
// same on every run.
//
// Coefficients live in box-id-indexed arrays [nbox + 1][S] (FP64); row nbox
// is all zero (the source of an absent M2L slot).  Multipoles are in units of
// their own box (mu = sum q rho(u)), locals ell with phi = (1/w) ell . rho(u),
// as in the uniform tree, so the same translation tables serve.  Potentials
// and fields leave the kernels in root units (phi * size, E * size^2).  Every
// kernel works in FP64 except, in the mixed form, the M2L (binary16 parts on
// the 16-bit matrix cores), the P2P pairs (FP32 on FP64 differences) and the
// P2M, L2P, P2L and M2P terms (FP32, summed in FP64).
#include <algorithm>

#include "harmonics.hpp"
#include <type_traits>

#include "kernels.hpp"

namespace fmm {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// LDS written by some lanes of a wave and read by others: the wave's own
// barrier with the fences that order its LDS accesses
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ tree build
__device__ __forceinline__ void box_coords(uint32_t code, int64_t &x, int64_t &y, int64_t &z) {
    x = compact3(code);
    y = compact3(code >> 1);
    z = compact3(code >> 2);
}

// closed cubes of boxes (la, a) and (lb, b) touch and neither contains the other
__device__ inline bool ad_adjacent(int la, uint32_t ca, int lb, uint32_t cb) {
    const bool af = la >= lb;  // a is the finer (or equal)
    const int k = af ? la - lb : lb - la;
    int64_t f[3], c[3];
    box_coords(af ? ca : cb, f[0], f[1], f[2]);
    box_coords(af ? cb : ca, c[0], c[1], c[2]);
    bool inside = true;
    for (int ax = 0; ax < 3; ++ax) {
        const int64_t lo = c[ax] << k, hi = ((c[ax] + 1) << k) - 1;
        if (f[ax] < lo - 1 || f[ax] > hi + 1) return false;
        if (f[ax] < lo || f[ax] > hi) inside = false;
    }
    return !inside;
}

// a box as its level and coordinates at that level (each below 2^10), for
// the list walks, which test one box against many: decoded once, compared
// in 32-bit arithmetic
struct AdBox {
    int l, x, y, z;
};
__device__ __forceinline__ AdBox ad_box(int l, uint32_t code) {
    return AdBox{l, (int)compact3(code), (int)compact3(code >> 1), (int)compact3(code >> 2)};
}
// ad_adjacent on decoded boxes
__device__ __forceinline__ bool ad_touch(const AdBox a, const AdBox b) {
    const bool af = a.l >= b.l;  // a is the finer (or equal)
    const int k = af ? a.l - b.l : b.l - a.l;
    const int f[3] = {af ? a.x : b.x, af ? a.y : b.y, af ? a.z : b.z};
    const int c[3] = {af ? b.x : a.x, af ? b.y : a.y, af ? b.z : a.z};
    bool inside = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int lo = c[ax] << k, hi = ((c[ax] + 1) << k) - 1;
        if (f[ax] < lo - 1 || f[ax] > hi + 1) return false;
        if (f[ax] < lo || f[ax] > hi) inside = false;
    }
    return !inside;
}

__global__ void k_ad_root(uint32_t n, uint32_t *code, uint32_t *ps, uint32_t *pe, int *parent) {
    code[0] = 0;
    ps[0] = 0;
    pe[0] = n;
    parent[0] = -1;
}

// The first sorted position whose key at the finest level Lf is >= x (x in
// [0, 8^Lf]): the table entry when x is a key of level cl, else a binary
// search of the sorted keys between the entries of x's level-cl key.
__device__ __forceinline__ uint32_t key_start(const KeyIndex &ki, uint64_t x) {
    const int sh = 3 * (ki.Lf - ki.cl);
    const uint64_t xc = x >> sh;
    uint32_t lo = ki.cstart[xc];
    if ((x & ((1ull << sh) - 1)) == 0) return lo;
    uint32_t hi = ki.cstart[xc + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)ki.skey[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Split decision and the non-empty children of the level's boxes [b0, b0+nb).
__global__ void k_ad_count(int64_t b0, int64_t nb, int l, int Lf, int leaf_max, const uint32_t *__restrict__ code,
                           const uint32_t *__restrict__ ps, const uint32_t *__restrict__ pe, const KeyIndex ki,
                           uint8_t *__restrict__ leaf, uint32_t *__restrict__ nchild, uint8_t *__restrict__ cmask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int64_t g = b0 + i;
    const bool split = pe[g] - ps[g] > (uint32_t)leaf_max && l < Lf;
    uint32_t k = 0, mask = 0;
    if (split) {
        const int sh = 3 * (Lf - l - 1);
        const uint64_t m0 = (uint64_t)code[g] << 3;
        uint32_t s = key_start(ki, m0 << sh);
        for (uint32_t c = 0; c < 8; ++c) {
            const uint32_t e = key_start(ki, (m0 + c + 1) << sh);
            if (e > s) {
                mask |= 1u << c;
                ++k;
            }
            s = e;
        }
    }
    leaf[g] = split ? 0 : 1;
    nchild[i] = k;
    cmask[g] = (uint8_t)mask;
}

// Append the children of level l's boxes at global ids next0 + coff[i] ...
__global__ void k_ad_children(int64_t b0, int64_t nb, int l, int Lf, int64_t next0, const KeyIndex ki,
                              const uint32_t *__restrict__ coff,
                              const uint8_t *__restrict__ cmask, uint32_t *__restrict__ code,
                              uint32_t *__restrict__ ps, uint32_t *__restrict__ pe, int *__restrict__ parent,
                              int *__restrict__ child) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int64_t g = b0 + i;
    const uint32_t mask = cmask[g];
    int64_t j = next0 + coff[i];
    const int sh = 3 * (Lf - l - 1);
    for (uint32_t c = 0; c < 8; ++c) {
        if (!((mask >> c) & 1u)) {
            child[8 * g + c] = -1;
            continue;
        }
        const uint64_t m = ((uint64_t)code[g] << 3) | c;
        code[j] = (uint32_t)m;
        ps[j] = key_start(ki, m << sh);
        pe[j] = key_start(ki, (m + 1) << sh);
        parent[j] = (int)g;
        child[8 * g + c] = (int)j;
        ++j;
    }
}

// Colleagues (the 27 same-level boxes at offsets -1..1, -1 if absent) of the
// level's boxes, by binary search in the level's Morton-sorted codes; one
// thread per (box, offset).
__global__ void k_ad_colleagues(int64_t b0, int64_t nb, int l, const uint32_t *__restrict__ code,
                                int *__restrict__ col) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 27 * nb) return;
    const int64_t g = b0 + i / 27;
    const int o = (int)(i % 27);
    int64_t x, y, z;
    box_coords(code[g], x, y, z);
    const int64_t side = (int64_t)1 << l;
    const int64_t sx = x + o % 3 - 1, sy = y + (o / 3) % 3 - 1, sz = z + o / 9 - 1;
    int r = -1;
    if (sx >= 0 && sy >= 0 && sz >= 0 && sx < side && sy < side && sz < side) {
        const uint32_t key = morton3((uint32_t)sx, (uint32_t)sy, (uint32_t)sz);
        int64_t lo = b0, hi = b0 + nb - 1;
        while (lo <= hi) {
            const int64_t mid = (lo + hi) >> 1;
            const uint32_t k = code[mid];
            if (k == key) {
                r = (int)mid;
                break;
            }
            if (k < key) lo = mid + 1;
            else hi = mid - 1;
        }
    }
    col[27 * g + o] = r;
}

// V as slots: for box g of level l >= 2 and class k (its coordinate parities),
// slot s of the class's 189 offsets holds the source box t + d if it exists
// (a child of one of the parent's colleagues), else -1; one thread per
// (box, slot).
__global__ void k_ad_vslots(int64_t b0, int64_t nb, const uint32_t *__restrict__ code,
                            const int *__restrict__ parent, const int *__restrict__ col,
                            const int *__restrict__ child, const int2 *__restrict__ cls,
                            int *__restrict__ vidx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)kOffsetsPerClass * nb) return;
    const int64_t bi = i / kOffsetsPerClass;
    const int s = (int)(i - bi * kOffsetsPerClass);
    const int64_t g = b0 + bi;
    int64_t tx, ty, tz;
    box_coords(code[g], tx, ty, tz);
    const int k = (int)((tx & 1) | ((ty & 1) << 1) | ((tz & 1) << 2));
    const int e = cls[k * kOffsetsPerClass + s].x;
    const int64_t sx = tx + (e & 15) - 4, sy = ty + ((e >> 4) & 15) - 4, sz = tz + ((e >> 8) & 15) - 4;
    int r = -1;
    if (sx >= 0 && sy >= 0 && sz >= 0) {
        const int64_t ox = (sx >> 1) - (tx >> 1), oy = (sy >> 1) - (ty >> 1), oz = (sz >> 1) - (tz >> 1);
        const int pc = col[27 * (int64_t)parent[g] + (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)];
        if (pc >= 0) r = child[8 * (int64_t)pc + ((sx & 1) | ((sy & 1) << 1) | ((sz & 1) << 2))];
    }
    vidx[i] = r;
}

// The parts of U and W (leaf g only) and of X (any box g) that come
// through colleague direction o (counts only when the item pointers are
// NULL).  o = 13 (the box itself): U = {g}.  Otherwise one walk over the
// colleagues o of g's proper ancestors (from the parent up) that are
// leaves: one touching g goes to U, one touching g's parent but not g to X.
// Then g's own colleague o: a leaf goes to U, a split one is opened depth
// first (touching leaves to U, touching split boxes opened, the rest to W).
__device__ void ad_uwx(int g, int o, bool lg_leaf, const int *lev, const uint32_t *code, const int *parent,
                       const int *col, const int *child, const uint8_t *leaf, int *u, int &nu, int *w, int &nw,
                       int *x, int &nx) {
    nu = nw = nx = 0;
    if (o == 13) {
        if (lg_leaf) {
            if (u) u[0] = g;
            nu = 1;
        }
        return;
    }
    const AdBox bg = ad_box(lev[g], code[g]);
    const int p = parent[g];
    if (p >= 0) {
        const AdBox bp = ad_box(lev[p], code[p]);
        for (int a = p; a >= 0; a = parent[a]) {
            const int c = col[27 * (int64_t)a + o];
            if (c < 0 || !leaf[c]) continue;
            const AdBox bc = ad_box(lev[c], code[c]);
            if (ad_touch(bg, bc)) {
                if (lg_leaf) {
                    if (u) u[nu] = c;
                    ++nu;
                }
            } else if (ad_touch(bp, bc)) {
                if (x) x[nx] = c;
                ++nx;
            }
        }
    }
    if (!lg_leaf) return;
    const int c = col[27 * (int64_t)g + o];
    if (c < 0) return;
    if (leaf[c]) {
        if (u) u[nu] = c;
        ++nu;
        return;
    }
    int stack[8 * (FMM_MAX_LEVEL + 1)];
    int sp = 0;
    for (int ch = 7; ch >= 0; --ch)
        if (child[8 * (int64_t)c + ch] >= 0) stack[sp++] = child[8 * (int64_t)c + ch];
    while (sp > 0) {
        const int d = stack[--sp];
        if (!ad_touch(bg, ad_box(lev[d], code[d]))) {
            if (w) w[nw] = d;
            ++nw;
        } else if (leaf[d]) {
            if (u) u[nu] = d;
            ++nu;
        } else {
            for (int ch = 7; ch >= 0; --ch)
                if (child[8 * (int64_t)d + ch] >= 0) stack[sp++] = child[8 * (int64_t)d + ch];
        }
    }
}

// One thread per (box, direction), i = 27 g + o.  pass 0: counts of U, W
// (leaves) and X (all boxes); pass 1: the items, at the scanned offsets
// (ou, ow, ox: the three runs of one scan, each taken from its first entry).
__global__ void k_ad_lists(int64_t nbox, int pass, const int *__restrict__ lev, const uint32_t *__restrict__ code,
                           const int *__restrict__ parent, const int *__restrict__ col,
                           const int *__restrict__ child, const uint8_t *__restrict__ leaf,
                           uint32_t *__restrict__ nu, uint32_t *__restrict__ nw, uint32_t *__restrict__ nx,
                           const uint32_t *__restrict__ ou, const uint32_t *__restrict__ ow,
                           const uint32_t *__restrict__ ox, int *__restrict__ iu, int *__restrict__ iw,
                           int *__restrict__ ix) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 27 * nbox) return;
    const int g = (int)(i / 27), o = (int)(i % 27);
    int a, b, c;
    if (pass == 0) {
        ad_uwx(g, o, leaf[g] != 0, lev, code, parent, col, child, leaf, nullptr, a, nullptr, b, nullptr, c);
        nu[i] = a;
        nw[i] = b;
        nx[i] = c;
    } else {
        ad_uwx(g, o, leaf[g] != 0, lev, code, parent, col, child, leaf, iu + (ou[i] - ou[0]), a,
               iw + (ow[i] - ow[0]), b, ix + (ox[i] - ox[0]), c);
    }
}

// Per-box list offsets from the per-(box, direction) scans: box g starts at
// its direction 0 (g = nbox: the totals).
__global__ void k_ad_box_offsets(int64_t nbox, const uint32_t *__restrict__ s27, uint32_t *__restrict__ ou,
                                 uint32_t *__restrict__ ow, uint32_t *__restrict__ ox) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g > nbox) return;
    const int64_t m = 27 * nbox;  // one scan of the U, W and X counts: run k starts at s27[k m]
    ou[g] = s27[27 * g];
    ow[g] = s27[m + 27 * g] - s27[m];
    ox[g] = s27[2 * m + 27 * g] - s27[2 * m];
}

// level of every box from the level offsets
__global__ void k_ad_levels(int64_t nbox, const int64_t *__restrict__ off, int nlev, int *__restrict__ lev) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nbox) return;
    int l = 0;
    for (int j = 1; j < nlev; ++j)
        if (g >= off[j]) l = j;
    lev[g] = l;
}

// Leaves in particle order: head[ps] = leaf id, compacted by a scan
__global__ void k_ad_heads(int64_t nbox, const uint8_t *__restrict__ leaf, const uint32_t *__restrict__ ps,
                           const uint32_t *__restrict__ pe, uint32_t *__restrict__ is_head,
                           int *__restrict__ head) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nbox || !leaf[g]) return;
    is_head[ps[g]] = 1u;
    head[ps[g]] = (int)g;
}
__global__ void k_ad_leaflist(int64_t n, const uint32_t *__restrict__ is_head, const uint32_t *__restrict__ hoff,
                              const int *__restrict__ head, const uint32_t *__restrict__ ps,
                              int *__restrict__ lbox, uint32_t *__restrict__ lstart, uint8_t *__restrict__ llev,
                              const int *__restrict__ lev) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (is_head[i]) {
        const uint32_t j = hoff[i];
        const int g = head[i];
        lbox[j] = g;
        lstart[j] = ps[g];
        llev[j] = (uint8_t)lev[g];
    }
    if (i == n - 1) lstart[hoff[n]] = (uint32_t)n;
}

// The fullest leaf: a block maximum over a grid stride, one atomic per block.
__global__ __launch_bounds__(256) void k_ad_leafmax(int64_t nleaf, const uint32_t *__restrict__ lstart,
                                                    unsigned int *__restrict__ mx) {
    __shared__ unsigned int red[256];
    unsigned int m = 0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < nleaf; j += (int64_t)gridDim.x * 256)
        m = max(m, lstart[j + 1] - lstart[j]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomic_max_shared(mx, red[0]);
}

// Work units: ceil(count / 64) per leaf (pass 0), then each unit's (leaf,
// first target) from the scanned counts (pass 1), in two orders: units for
// P2P and units_m for M2P.  The counts are laid out as 2 kAdUnitClasses runs
// of nleaf (the P2P classes, then the M2P classes), by the weight of a full
// unit of the leaf, so that one scan orders each copy heaviest class first
// (about a longest-first schedule, which a sort would refine by ~1%): the
// heaviest waves then start with the grid instead of wherever the leaf order
// puts them, and the kernel does not end on a late heavy wave.  P2P weight:
// the unit's pairs, its targets times the sources of U; M2P weight: its
// rounds of W boxes, |W| over the lane groups of the unit, times 2^12.
// Classes: weight at least 2^19, 2^18, ..., 2^13, then the rest.
__global__ void k_ad_units(int64_t nleaf, int pass, const uint32_t *__restrict__ lstart,
                           const int *__restrict__ lbox, const uint32_t *__restrict__ ou,
                           const uint32_t *__restrict__ ow, const int *__restrict__ iu,
                           const uint32_t *__restrict__ ps, const uint32_t *__restrict__ pe,
                           uint32_t *__restrict__ cnt, const uint32_t *__restrict__ uoff,
                           int2 *__restrict__ units, int2 *__restrict__ units_m) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nleaf) return;
    const uint32_t np = lstart[j + 1] - lstart[j], m = (np + 63) / 64;
    const int64_t half = (int64_t)kAdUnitClasses * nleaf;
    if (pass == 0) {
        const int g = lbox[j];
        const uint32_t nt = min(np, 64u);
        uint64_t src = 0;
        for (uint32_t e = ou[g]; e < ou[g + 1]; ++e) {
            const int c = iu[e];
            src += pe[c] - ps[c];
        }
        uint32_t t = 4;  // the lane groups of k_ad_m2p: 64 / T, T = max(4, nt rounded up to a power of 2)
        while (t < nt && t < 64) t <<= 1;
        const uint32_t groups = 64 / t;
        const uint64_t weight[2] = {(uint64_t)nt * src, (uint64_t)((ow[g + 1] - ow[g] + groups - 1) / groups) << 12};
#pragma unroll
        for (int kind = 0; kind < 2; ++kind) {
            int cls = 0;
            while (cls < kAdUnitClasses - 1 && weight[kind] < (1ull << (19 - cls))) ++cls;
            for (int k = 0; k < kAdUnitClasses; ++k) cnt[kind * half + k * nleaf + j] = k == cls ? m : 0;
        }
        return;
    }
#pragma unroll
    for (int kind = 0; kind < 2; ++kind) {
        // the class is the run whose count is set (a leaf has m >= 1)
        int cls = 0;
        while (cls < kAdUnitClasses - 1 && cnt[kind * half + cls * nleaf + j] == 0) ++cls;
        const uint32_t base = uoff[kind * half + cls * nleaf + j] - (kind ? uoff[half] : 0u);
        int2 *dst = kind ? units_m : units;
        for (uint32_t k = 0; k < m; ++k) dst[base + k] = make_int2((int)j, (int)(64 * k));
    }
}

// Work counts: [0] ordered P2P pairs (self pairs included), [1] V entries,
// [2] (particle, box) pairs of W, [3] of X.
__global__ void k_ad_counts(int64_t nbox, int64_t box2, const uint8_t *__restrict__ leaf,
                            const uint32_t *__restrict__ ps, const uint32_t *__restrict__ pe,
                            const uint32_t *__restrict__ ou, const int *__restrict__ iu,
                            const uint32_t *__restrict__ ow, const uint32_t *__restrict__ ox,
                            const int *__restrict__ ix, const int *__restrict__ vidx,
                            unsigned long long *__restrict__ out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nbox) return;
    const unsigned long long ng = pe[g] - ps[g];
    unsigned long long u = 0, v = 0, xs = 0;
    if (leaf[g])
        for (uint32_t e = ou[g]; e < ou[g + 1]; ++e) u += pe[iu[e]] - ps[iu[e]];
    if (g >= box2)
        for (int s = 0; s < kOffsetsPerClass; ++s) v += vidx[kOffsetsPerClass * (g - box2) + s] >= 0;
    for (uint32_t e = ox[g]; e < ox[g + 1]; ++e) xs += pe[ix[e]] - ps[ix[e]];
    if (u) atomicAdd(out, u * ng);
    if (v) atomicAdd(out + 1, v);
    if (ow[g + 1] > ow[g]) atomicAdd(out + 2, ng * (ow[g + 1] - ow[g]));
    if (xs) atomicAdd(out + 3, xs);
}

// Sorted records relative to each particle's leaf (leaf units, FP64); the
// leaf of sorted position i is the last leaf head at or before i.
template <typename Tin>
__global__ void k_ad_records(int64_t n, const uint32_t *__restrict__ hoff, const int *__restrict__ lbox,
                             const int *__restrict__ lev, const uint32_t *__restrict__ code,
                             const uint32_t *__restrict__ perm, const Tin *__restrict__ pos, double lo0,
                             double lo1, double lo2, double inv_size, double4 *__restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int g = lbox[hoff[i + 1] - 1];
    const int l = lev[g];
    int64_t bx, by, bz;
    box_coords(code[g], bx, by, bz);
    const double sc = (double)((int64_t)1 << l) * inv_size;
    const uint32_t o = perm[i];
    double4 r;
    r.x = ((double)pos[3 * (size_t)o] - lo0) * sc - ((double)bx + 0.5);
    r.y = ((double)pos[3 * (size_t)o + 1] - lo1) * sc - ((double)by + 0.5);
    r.z = ((double)pos[3 * (size_t)o + 2] - lo2) * sc - ((double)bz + 0.5);
    r.w = 0.0;
    rec[i] = r;
}

// --------------------------------------------------------------- evaluate
// centre of box (l1, c1) minus centre of box (l2, c2), in units of the
// width of level lu (exact in FP64: dyadic rationals)
__device__ inline void ad_centre_diff(int l1, uint32_t c1, int l2, uint32_t c2, int lu, double &dx, double &dy,
                                      double &dz) {
    int64_t a[3], b[3];
    box_coords(c1, a[0], a[1], a[2]);
    box_coords(c2, b[0], b[1], b[2]);
    const double s1 = ldexp(1.0, lu - l1), s2 = ldexp(1.0, lu - l2);
    dx = ((double)a[0] + 0.5) * s1 - ((double)b[0] + 0.5) * s2;
    dy = ((double)a[1] + 0.5) * s1 - ((double)b[1] + 0.5) * s2;
    dz = ((double)a[2] + 0.5) * s1 - ((double)b[2] + 0.5) * s2;
}

// Regular solid harmonics times a seed, s R_n^m(x) for 0 <= m <= n < N, by
// the recurrences of regular_rho (R_m^m = -(x - iy)/(2m) R_{m-1}^{m-1},
// R_{m+1}^m = z R_m^m, (n-m)(n+m) R_n^m = (2n-1) z R_{n-1}^m - r^2
// R_{n-2}^m, linear in the seed), unrolled at compile time and visited
// column by column: f(n, m, re, im), im = 0 for m = 0.
template <int N, typename R, typename F>
__device__ __forceinline__ void regular_each(R x, R y, R z, R seed, F &&f) {
    const R r2 = x * x + y * y + z * z;
    R dr = seed, di = R(0);  // s R_m^m
#pragma unroll
    for (int m = 0; m < N; ++m) {
        if (m > 0) {
            const R inv = R(-1) / R(2 * m);
            const R nr = (dr * x + di * y) * inv, ni = (di * x - dr * y) * inv;
            dr = nr;
            di = ni;
        }
        R ar = dr, ai = di, br = R(0), bi = R(0);
#pragma unroll
        for (int n = m; n < N; ++n) {
            R cr = ar, ci = ai;
            if (n == m + 1) {
                cr = z * ar;
                if (m > 0) ci = z * ai;
            } else if (n > m + 1) {
                const R inv = R(1) / R((n - m) * (n + m)), h = R(2 * n - 1) * inv * z, c = inv * r2;
                cr = h * ar - c * br;
                if (m > 0) ci = h * ai - c * bi;
            }
            if (n > m) {
                br = ar;
                bi = ai;
                ar = cr;
                ai = ci;
            }
            f(n, m, cr, m > 0 ? ci : R(0));
        }
    }
}

// P2M at the leaves: mu(g) = sum_j q_j rho(u_j), leaf units; one block of 64
// per leaf, B particles' harmonics (times their charges) at a time as LDS
// rows, summed in FP64 coefficient by coefficient over the rows filled.  R:
// the arithmetic of the harmonics (FP32 in the mixed form, the leaf-relative
// position rounded once).  adj = 1: the
// transpose of L2P (the weights' sum times 2^l, the leaf's root-unit factor).
template <int P, typename R>
__global__ __launch_bounds__(64) void k_ad_p2m(const int *__restrict__ lbox, const uint32_t *__restrict__ lstart,
                                               const uint8_t *__restrict__ llev, int adj,
                                               const double4 *__restrict__ rec, double *__restrict__ M) {
    constexpr int P2 = P * P, S = coef_stride(P), NC = (S + 63) / 64;
    // rows of at most ~17 KB
    constexpr int B0 = P <= 5 ? 64 : P <= 8 ? 32 : P <= 11 ? 16 : 8, B = sizeof(R) == 4 && B0 < 64 ? 2 * B0 : B0;
    __shared__ R rows[B][P2 + 1];
    const int j = blockIdx.x, t = threadIdx.x;
    const uint32_t s0 = lstart[j], s1 = lstart[j + 1];
    double acc[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) acc[a] = 0.0;
    for (uint32_t b0 = s0; b0 < s1; b0 += B) {
        __syncthreads();
        if (t < B && b0 + t < s1) {
            R *row = rows[t];
            const double4 r = rec[b0 + t];
            regular_each<P>((R)r.x, (R)r.y, (R)r.z, (R)r.w, [&](int n, int m, R re, R im) {
                if (m == 0) {
                    row[n * n] = re;
                } else {
                    row[n * n + 2 * m - 1] = re;
                    row[n * n + 2 * m] = im;
                }
            });
        }
        __syncthreads();
        const int nr = (int)min((uint32_t)B, s1 - b0);
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            const int c = t + 64 * a;
            if (c < P2)
                for (int k = 0; k < nr; ++k) acc[a] += (double)rows[k][c];
        }
    }
    const int g = lbox[j];
    const double f = adj ? ldexp(1.0, (int)llev[j]) : 1.0;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
        const int c = t + 64 * a;
        if (c < S) M[(size_t)g * S + c] = c < P2 ? acc[a] * f : 0.0;
    }
}

// M2M for the split boxes of one level: mu(g) = sum_c A_c mu(child c)
// (tab [8][p^2][p^2] input-major, [c][in][out]).  A block takes BX
// consecutive boxes of the level, so that each table entry read from L2
// serves BX boxes (one box a block read the whole 8 p^4 table per box); its
// threads are (output o, K part kg), KG parts of the p^2 inputs per output,
// whose partial sums are joined through LDS in kg order.
template <int P>
__global__ __launch_bounds__(256) void k_ad_m2m(int64_t b0, int64_t nb, const uint8_t *__restrict__ leaf,
                                                const int *__restrict__ child, const double *__restrict__ tab,
                                                double *__restrict__ M) {
    constexpr int P2 = P * P, S = coef_stride(P);
    constexpr int KG = P2 > 128 ? 1 : (P2 > 64 ? 2 : 4);
    constexpr int BX0 = 4096 / (8 * P2), BX = BX0 < 1 ? 1 : (BX0 > 8 ? 8 : BX0);
    constexpr int KL = (P2 + KG - 1) / KG;  // inputs per part
    __shared__ double in[BX][8][P2];
    __shared__ double part[KG][BX][P2];
    __shared__ int has[BX][8];
    const int64_t g0 = b0 + (int64_t)blockIdx.x * BX;
    const int nbx = (int)min((int64_t)BX, b0 + nb - g0);
    const int tid = threadIdx.x;
    for (int i = tid; i < BX * 8 * P2; i += 256) {
        const int bx = i / (8 * P2), r = i - bx * 8 * P2, c = r / P2, k = r - c * P2;
        int ch = -1;
        if (bx < nbx && !leaf[g0 + bx]) ch = child[8 * (g0 + bx) + c];
        in[bx][c][k] = ch >= 0 ? M[(size_t)ch * S + k] : 0.0;
    }
    for (int i = tid; i < BX * 8; i += 256) {
        const int bx = i >> 3, c = i & 7;
        has[bx][c] = bx < nbx && !leaf[g0 + bx] && child[8 * (g0 + bx) + c] >= 0;
    }
    __syncthreads();
    const int o = tid % P2, kg = tid / P2;
    if (kg < KG) {
        double v[BX];
#pragma unroll
        for (int bx = 0; bx < BX; ++bx) v[bx] = 0.0;
        const int k0 = kg * KL, k1 = min(P2, k0 + KL);
        for (int c = 0; c < 8; ++c) {
            bool any = false;
#pragma unroll
            for (int bx = 0; bx < BX; ++bx) any |= has[bx][c] != 0;
            if (!any) continue;
            const double *tc = tab + (size_t)c * P2 * P2 + o;
            for (int k = k0; k < k1; ++k) {
                const double a = tc[(size_t)k * P2];
#pragma unroll
                for (int bx = 0; bx < BX; ++bx) v[bx] = __builtin_fma(a, in[bx][c][k], v[bx]);
            }
        }
#pragma unroll
        for (int bx = 0; bx < BX; ++bx) part[kg][bx][o] = v[bx];
    }
    __syncthreads();
    for (int i = tid; i < BX * S; i += 256) {
        const int bx = i / S, oo = i - bx * S;
        if (bx >= nbx || leaf[g0 + bx]) continue;
        double v = 0.0;
        if (oo < P2)
#pragma unroll
            for (int q = 0; q < KG; ++q) v += part[q][bx][oo];
        M[(size_t)(g0 + bx) * S + oo] = v;
    }
}

// L2L into the boxes of one level (>= 3): ell(g) += B_c ell(parent)
template <int P>
__global__ __launch_bounds__(256) void k_ad_l2l(int64_t b0, const uint32_t *__restrict__ code,
                                                const int *__restrict__ parent, const double *__restrict__ tab,
                                                double *__restrict__ Lc) {
    constexpr int P2 = P * P, S = coef_stride(P);
    __shared__ double in[P2];
    const int64_t g = b0 + blockIdx.x;
    const int pa = parent[g];
    for (int k = threadIdx.x; k < P2; k += 256) in[k] = Lc[(size_t)pa * S + k];
    __syncthreads();
    const uint32_t cd = code[g];
    const int c = (int)(cd & 7u);  // the child octant: bit 0 x, 1 y, 2 z of the Morton code
    for (int o = threadIdx.x; o < P2; o += 256) {
        double v = 0.0;
        const double *tc = tab + (size_t)c * P2 * P2 + o;
        for (int k = 0; k < P2; ++k) v += tc[(size_t)k * P2] * in[k];
        Lc[(size_t)g * S + o] += v;
    }
}

// L2P at the leaves, outputs in root units (phi * 2^l, E * 4^l).  adj = 1:
// the transpose of P2M and its position derivative (phi, E * 2^l).  R: the
// arithmetic of the evaluation (FP32 in the mixed form: the local
// expansion and the leaf-relative position rounded once).
template <int P, typename R>
__global__ __launch_bounds__(64) void k_ad_l2p(const int *__restrict__ lbox, const uint32_t *__restrict__ lstart,
                                               const uint8_t *__restrict__ llev, int adj,
                                               const double4 *__restrict__ rec, const double *__restrict__ Lc,
                                               double4 *__restrict__ out) {
    using V = typename std::conditional<sizeof(R) == 4, float4, double4>::type;
    constexpr int P2 = P * P, S = coef_stride(P);
    __shared__ R ell[P2];
    __shared__ V coef[P2];
    const int j = blockIdx.x;
    const int g = lbox[j];
    for (int c = threadIdx.x; c < P2; c += 64) ell[c] = (R)Lc[(size_t)g * S + c];
    __syncthreads();
    for (int c = threadIdx.x; c < P2; c += 64) coef[c] = l2p_coef<R, V>(ell, P, c);
    __syncthreads();
    const double s1 = ldexp(1.0, (1 - adj) * (int)llev[j]), s2 = ldexp(1.0, (2 - adj) * (int)llev[j]);
    for (uint32_t i = lstart[j] + threadIdx.x; i < lstart[j + 1]; i += 64) {
        __asm__ volatile("" ::: "memory");
        const double4 r = rec[i];
        R phi, gx, gy, gz;
        l2p_point<P, R, V>(coef, (R)r.x, (R)r.y, (R)r.z, phi, gx, gy, gz);
        out[i] = make_double4((double)phi * s1, -(double)gx * s2, -(double)gy * s2, -(double)gz * s2);
    }
}

// Irregular solid harmonics I_n^m(y) for 0 <= m <= n <= N (complex, as in
// the translation operators: I_0^0 = 1/r, I_m^m = -(2m-1) (x+iy)/r^2
// I_{m-1}^{m-1}, I_{m+1}^m = (2m+1) z/r^2 I_m^m, r^2 I_n^m = (2n-1) z
// I_{n-1}^m - (n-m-1)(n+m-1) I_{n-2}^m), visited column by column: f(n, m,
// re, im) for every pair, in the arithmetic type R of the position.
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int N, typename R, typename F>
__device__ __forceinline__ void irregular_each(R x, R y, R z, F &&f) {
    const R r2 = x * x + y * y + z * z, ir2 = R(1) / r2, zr = z * ir2;
    R dr = sqrt(ir2), di = R(0);  // I_m^m
#pragma unroll
    for (int m = 0; m <= N; ++m) {
        if (m > 0) {
            const R k = -R(2 * m - 1) * ir2;
            const R nr = k * (x * dr - y * di), ni = k * (x * di + y * dr);
            dr = nr;
            di = ni;
        }
        // column m; the imaginary parts of column 0 are zero and not formed
        R ar = dr, ai = di, br = R(0), bi = R(0);
#pragma unroll
        for (int n = m; n <= N; ++n) {
            R cr = ar, ci = ai;
            if (n == m + 1) {
                const R h = R(2 * m + 1) * zr;
                cr = h * ar;
                if (m > 0) ci = h * ai;
            } else if (n > m + 1) {
                const R h = R(2 * n - 1) * zr, c = R((n - m - 1) * (n + m - 1)) * ir2;
                cr = h * ar - c * br;
                if (m > 0) ci = h * ai - c * bi;
            }
            if (n > m) {
                br = ar;
                bi = ai;
                ar = cr;
                ai = ci;
            }
            f(n, m, cr, m > 0 ? ci : R(0));
        }
    }
}

// P2L over X: for every box g, ell(g) = sum over the leaves c of X(g) of the
// local expansion of each particle of c: the complex local coefficient of a
// charge q at y (g units) is q I_n^m(y), i.e. ell_c = 2 q Re, ell_s = -2 q Im.
// Every box's row is written (zero for an empty X), so this pass also clears
// the locals before M2L and L2L add to them.  One wave per box: the
// particles of X(g) are taken as one sequence (up to 64 list entries at a
// time, offsets by a wave scan, each lane finding its entry by bisection),
// B of them at a time each expanded by one lane into an LDS row, and the
// rows summed coefficient by coefficient.  R is the arithmetic of the
// expansion (FP32 in the mixed form, the offset formed in FP64 and rounded
// once); the rows are summed in FP64.
template <int P, typename R>
__global__ __launch_bounds__(64) void k_ad_p2l(const uint32_t *__restrict__ ox, const int *__restrict__ ix,
                                               const int *__restrict__ lev, const uint32_t *__restrict__ code,
                                               const uint32_t *__restrict__ ps, const uint32_t *__restrict__ pe,
                                               int adj, const double4 *__restrict__ rec, double *__restrict__ Lc) {
    constexpr int P2 = P * P, S = coef_stride(P), NC = (P2 + 63) / 64;
    // rows of at most ~17 KB (2 waves per SIMD)
    constexpr int B = (P <= 8 ? 32 : (P <= 11 ? 16 : 8)) * (int)(sizeof(double) / sizeof(R));
    __shared__ R rows[B][P2 + 1];
    __shared__ double4 frame[64];
    __shared__ uint32_t first[64], off[65];
    const int g = blockIdx.x, t = threadIdx.x;
    const uint32_t x0 = ox[g], x1 = ox[g + 1];
    const int lg = lev[g];
    const uint32_t cg = code[g];
    double acc[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) acc[a] = 0.0;
    for (uint32_t e0 = x0; e0 < x1; e0 += 64) {
        const int nb = (int)min(64u, x1 - e0);
        uint32_t cnt = 0;
        __syncthreads();  // the previous batch's tables have been read
        if (t < nb) {
            const int c = ix[e0 + t];
            const int lc = lev[c];
            double cx, cy, cz;
            ad_centre_diff(lc, code[c], lg, cg, lg, cx, cy, cz);
            frame[t] = make_double4(cx, cy, cz, ldexp(1.0, lg - lc));
            first[t] = ps[c];
            cnt = pe[c] - ps[c];
        }
        uint32_t incl = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t v = __shfl_up(incl, d);
            if (t >= d) incl += v;
        }
        off[t + 1] = incl;
        if (t == 0) off[0] = 0;
        const uint32_t total = __shfl(incl, 63);
        __syncthreads();
        for (uint32_t f0 = 0; f0 < total; f0 += B) {
            __syncthreads();  // the previous rows have been summed
            if (t < B) {
                R *row = rows[t];
                const uint32_t f = f0 + t;
                if (f < total) {
                    int lo = 0, hi = nb - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (off[mid] <= f) lo = mid;
                        else hi = mid - 1;
                    }
                    const double4 fr = frame[lo];
                    const double4 v = rec[first[lo] + (f - off[lo])];
                    const R q = (R)v.w;
                    irregular_each<P - 1>((R)(fr.x + fr.w * v.x), (R)(fr.y + fr.w * v.y), (R)(fr.z + fr.w * v.z),
                                          [&](int n, int m, R re, R im) {
                                              if (m == 0) {
                                                  row[n * n] = q * re;
                                              } else {
                                                  row[n * n + 2 * m - 1] = R(2) * q * re;
                                                  row[n * n + 2 * m] = -R(2) * q * im;
                                              }
                                          });
                } else {
                    for (int k = 0; k < P2; ++k) row[k] = R(0);
                }
            }
            __syncthreads();
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                const int k = t + 64 * a;
                if (k < P2)
                    for (int r = 0; r < B; ++r) acc[a] += (double)rows[r][k];
            }
        }
    }
    const double f = adj ? ldexp(1.0, lg) : 1.0;  // adj = 1: the transpose of M2P
#pragma unroll
    for (int a = 0; a < NC; ++a) {
        const int k = t + 64 * a;
        if (k < P2) Lc[(size_t)g * S + k] = acc[a] * f;
    }
}

// M2P over W at the leaves: the field of the truncated multipole of each w in
// W(g) at g's particles.  With M_n^m = mu_c + i mu_s (M_n^{-m} = (-1)^m
// conj) and y the particle relative to w's centre (w units), the degree-0
// and degree-1 coefficients of the local expansion at the particle are
//   L_0^0 = sum M_n^m I_n^m,  L_1^l = -sum M_n^m I_{n+1}^{m+l},
// and phi = L_0^0 / w, grad = (-Re L_1^1, -Im L_1^1, L_1^0) / w^2.
// Added into out (root units: phi * 2^l_w, E * 4^l_w; adj = 1, the
// transpose of P2L and its position derivative: phi, E * 2^l_w).  One wave per unit
// of up to 64 targets (the P2P units): the targets take T = 2^LT lanes, and
// the 64 / T lane groups take the boxes of W(g) in turn, each staging its
// box's multipole in LDS; the groups' sums are joined by shuffles.  R is
// the arithmetic of one box's terms (FP32 in the mixed form: multipole and
// offset rounded once); the boxes' sums are added in FP64.
template <int P, int LT, typename R>
__device__ __forceinline__ void ad_m2p_unit(R (*mus)[P * P], int lane, int adj, int g, int lg, uint32_t cg,
                                            uint32_t t0, uint32_t nt, uint32_t w0, uint32_t w1,
                                            const int *__restrict__ iw,
                                            const int *__restrict__ lev, const uint32_t *__restrict__ code,
                                            const double4 *__restrict__ rec, const double *__restrict__ M,
                                            double4 *__restrict__ out) {
    constexpr int P2 = P * P, S = coef_stride(P), T = 1 << LT, G = 64 >> LT;
    const int slot = lane & (T - 1), grp = lane >> LT;
    const bool live = (uint32_t)slot < nt;
    const double4 r = live ? rec[t0 + slot] : make_double4(0.0, 0.0, 0.0, 0.0);
    double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    R *const mu = mus[grp];
    for (uint32_t e0 = w0; e0 < w1; e0 += G) {
        const uint32_t e = e0 + grp;
        const bool has = e < w1;
        const int w = has ? iw[e] : 0;
        wave_sync();  // the previous round's multipoles have been read
        if (has)
            for (int c = slot; c < P2; c += T) mu[c] = (R)M[(size_t)w * S + c];
        wave_sync();
        if (!has) continue;
        const int lw = lev[w];
        double cx, cy, cz;
        ad_centre_diff(lg, cg, lw, code[w], lw, cx, cy, cz);
        const double sc = ldexp(1.0, lw - lg);
        // l00: L_0^0 = sum over n < P of M_n^m I_n^m with its conjugate
        // partner (m > 0 terms twice), l10: -L_1^0, the same over M_{n-1}^m,
        // l11: L_1^1 = -sum M_{n-1}^{m-1} I_n^m (m >= 1) + conj(M_{n-1}^{m+1}
        // I_n^m) (the terms of order -(m+1)).  Coefficients outside
        // 0 <= m' <= n' < P are zero and skipped at compile time; the m = 0
        // and m > 0 parts of l00 and l10 are kept apart, so that the factor 2
        // is applied once.
        R l00 = R(0), l00m = R(0), l10 = R(0), l10m = R(0), l11r = R(0), l11i = R(0);
        irregular_each<P>((R)(cx + sc * r.x), (R)(cy + sc * r.y), (R)(cz + sc * r.z), [&](int n, int m, R ir, R ii) {
            auto re_of = [&](int nn, int mm) { return mu[mm == 0 ? nn * nn : nn * nn + 2 * mm - 1]; };
            auto im_of = [&](int nn, int mm) { return mu[nn * nn + 2 * mm]; };
            // acc += Re(M_nn^mm I_n^m)
            auto add_re = [&](R &acc, int nn, int mm) {
                acc = fma_r(re_of(nn, mm), ir, acc);
                if (mm > 0) acc = fma_r(-im_of(nn, mm), ii, acc);
            };
            if (n < P) add_re(m == 0 ? l00 : l00m, n, m);
            if (n >= 1 && m <= n - 1) add_re(m == 0 ? l10 : l10m, n - 1, m);
            if (n >= 1 && m >= 1) {  // l11 -= M_{n-1}^{m-1} I
                const R mr = re_of(n - 1, m - 1);
                l11r = fma_r(-mr, ir, l11r);
                l11i = fma_r(-mr, ii, l11i);
                if (m - 1 > 0) {
                    const R mi = im_of(n - 1, m - 1);
                    l11r = fma_r(mi, ii, l11r);
                    l11i = fma_r(-mi, ir, l11i);
                }
            }
            if (n >= 1 && m + 1 <= n - 1) {  // l11 += conj(M_{n-1}^{m+1} I)
                const R mr = re_of(n - 1, m + 1), mi = im_of(n - 1, m + 1);
                l11r = fma_r(mr, ir, l11r);
                l11i = fma_r(-mi, ir, l11i);
                if (m > 0) {  // I_n^0 is real
                    l11r = fma_r(-mi, ii, l11r);
                    l11i = fma_r(-mr, ii, l11i);
                }
            }
        });
        l00 += R(2) * l00m;
        l10 = -(l10 + R(2) * l10m);
        const double s1 = ldexp(1.0, (1 - adj) * lw), s2 = ldexp(1.0, (2 - adj) * lw);
        phi += (double)l00 * s1;
        ex += (double)l11r * s2;
        ey += (double)l11i * s2;
        ez -= (double)l10 * s2;
    }
#pragma unroll
    for (int d = 32; d >= T; d >>= 1) {
        phi += __shfl_xor(phi, d);
        ex += __shfl_xor(ex, d);
        ey += __shfl_xor(ey, d);
        ez += __shfl_xor(ez, d);
    }
    if (live && grp == 0) {
        double4 o = out[t0 + slot];
        o.x += phi;
        o.y += ex;
        o.z += ey;
        o.w += ez;
        out[t0 + slot] = o;
    }
}

// at most 16 lane groups (4 lanes per unit target at least), so that the
// staged multipoles stay within 32 KB at p = 16
template <int P, typename R>
__global__ __launch_bounds__(64) void k_ad_m2p(const uint32_t *__restrict__ nunits, const int2 *__restrict__ units,
                                               int adj, const int *__restrict__ lbox, const uint32_t *__restrict__ lstart,
                                               const uint32_t *__restrict__ ow, const int *__restrict__ iw,
                                               const int *__restrict__ lev, const uint32_t *__restrict__ code,
                                               const double4 *__restrict__ rec, const double *__restrict__ M,
                                               double4 *__restrict__ out) {
    __shared__ R mus[16][P * P];
    if (blockIdx.x >= *nunits) return;
    const int2 un = units[blockIdx.x];
    const int j = un.x;
    const int g = lbox[j];
    const uint32_t w0 = ow[g], w1 = ow[g + 1];
    if (w0 == w1) return;
    const int lane = threadIdx.x;
    const uint32_t t0 = lstart[j] + (uint32_t)un.y, nt = min(64u, lstart[j + 1] - t0);
    int lt = 2;  // log2 T, at least 2
    while ((1u << lt) < nt && lt < 6) ++lt;
#define AD_M2P_CASE(K)                                                                                          \
    case K:                                                                                                     \
        ad_m2p_unit<P, K, R>(mus, lane, adj, g, lev[g], code[g], t0, nt, w0, w1, iw, lev, code, rec, M, out);     \
        break;
    switch (lt) { AD_M2P_CASE(2) AD_M2P_CASE(3) AD_M2P_CASE(4) AD_M2P_CASE(5) AD_M2P_CASE(6) }
#undef AD_M2P_CASE
}

// One pair of the FP64 near field: rsqrt by the hardware estimate and one
// Newton step (relative error near 2^-52); a coincident source (r = 0,
// which includes the target itself) adds nothing when SELF.
template <bool SELF>
__device__ __forceinline__ void ad_pair(double xi, double yi, double zi, const double4 s, double &phi,
                                        double &ex, double &ey, double &ez) {
    const double dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
    double r2 = dx * dx;
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

// The mixed form's pair: the FP64 difference rounded once to FP32 (both
// points in the target leaf's frame, so it carries no cancellation against
// absolute positions), then the FP32 arithmetic of the uniform tree's mixed
// P2P with the hardware reciprocal square root.
template <bool SELF>
__device__ __forceinline__ void ad_pair32(double xi, double yi, double zi, const double4 s, float &phi, float &ex,
                                          float &ey, float &ez) {
    const float dx = (float)(xi - s.x), dy = (float)(yi - s.y), dz = (float)(zi - s.z);
    float r2 = dx * dx;
    r2 = __builtin_fmaf(dy, dy, r2);
    r2 = __builtin_fmaf(dz, dz, r2);
    float y = __builtin_amdgcn_rsqf(r2);
    if (SELF) y = r2 > 0.0f ? y : 0.0f;
    const float qr = (float)s.w * y;
    phi += qr;
    const float qr3 = qr * (y * y);
    ex = __builtin_fmaf(qr3, dx, ex);
    ey = __builtin_fmaf(qr3, dy, ey);
    ez = __builtin_fmaf(qr3, dz, ez);
}

// P2P over U at the leaves (FP64), one wave per unit of up to 64 targets of
// one leaf (a leaf of more than 64 particles gives several units, so that
// the work of the fullest leaves spreads over several waves).  The unit's
// targets take T lanes, two per lane (T = half the count, rounded up), and
// the 64 / T lane groups split every source tile, their sums joined through
// LDS in group order at the end.  The sources of U(g) are taken as one sequence, up to
// 64 list entries at a time: each lane holds one entry's particle range and
// its frame change (c_c - c_g)/w_g + u 2^(l_g - l_c) (exact scaling, one
// rounding), a wave scan of the counts gives the entries' offsets, and the
// sequence is staged in tiles of 64 in the wave's LDS (the last one padded
// with far, uncharged points), each lane finding its entry by bisection.  A
// coincident source, the target itself included, adds nothing.  Root units
// out.
constexpr int kAdP2PWaves = 4;
struct AdP2PShared {
    double4 tile[64];
    double4 frame[64];    // (cx, cy, cz, scale) of a batch's entries
    uint32_t first[64];   // first particle of each entry
    uint32_t off[65];     // exclusive offsets of the entries, total last
};

// FUSE (1: FP32, 2: FP64 caller data): each target's sums go through the
// combine with its far field (c) into the caller's order instead of out.
// F32 (the mixed form): the pairs in FP32 (ad_pair32), each tile's partial
// sums merged into the FP64 sums.
template <int FUSE, bool F32>
__device__ __forceinline__ void ad_p2p_unit(AdP2PShared &sh, int lane, int g, int lg, uint32_t cg, uint32_t t0,
                                            uint32_t nt, uint32_t u0, uint32_t u1, const int *__restrict__ iu,
                                            const int *__restrict__ lev, const uint32_t *__restrict__ code,
                                            const uint32_t *__restrict__ ps, const uint32_t *__restrict__ pe,
                                            const double4 *__restrict__ rec, double4 *__restrict__ out,
                                            const Combine &c) {
    // T lanes hold the unit's targets, two per lane (slot and slot + T);
    // G = 64 / T groups of them split every source tile; lanes past G T idle
    const int T = (int)((nt + 1) / 2), G = 64 / T;
    const int grp = lane / T, slot = lane - grp * T;
    const bool act = grp < G;
    const double s1 = ldexp(1.0, lg), s2 = s1 * s1;
    const bool live0 = act && (uint32_t)slot < nt, live1 = act && (uint32_t)(slot + T) < nt;
    const double4 r0 = live0 ? rec[t0 + slot] : make_double4(0.0, 0.0, 0.0, 0.0);
    const double4 r1 = live1 ? rec[t0 + slot + T] : make_double4(0.0, 0.0, 0.0, 0.0);
    double phi0 = 0.0, ex0 = 0.0, ey0 = 0.0, ez0 = 0.0, phi1 = 0.0, ex1 = 0.0, ey1 = 0.0, ez1 = 0.0;
    for (uint32_t e0 = u0; e0 < u1; e0 += 64) {
        const int nb = (int)min(64u, u1 - e0);
        uint32_t cnt = 0;
        wave_sync();  // the previous batch's tables have been read
        if (lane < nb) {
            const int c = iu[e0 + lane];
            const int lc = lev[c];
            double cx, cy, cz;
            ad_centre_diff(lc, code[c], lg, cg, lg, cx, cy, cz);
            sh.frame[lane] = make_double4(cx, cy, cz, ldexp(1.0, lg - lc));
            sh.first[lane] = ps[c];
            cnt = pe[c] - ps[c];
        }
        uint32_t incl = cnt;  // inclusive scan over the lanes
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        sh.off[lane + 1] = incl;
        if (lane == 0) sh.off[0] = 0;
        const uint32_t total = __shfl(incl, 63);
        wave_sync();
        for (uint32_t f0 = 0; f0 < total; f0 += 64) {
            const uint32_t f = f0 + lane;
            double4 src = make_double4(1e3, 1e3, 1e3, 0.0);
            if (f < total) {
                int lo = 0, hi = nb - 1;  // the entry k with off[k] <= f < off[k + 1]
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sh.off[mid] <= f) lo = mid;
                    else hi = mid - 1;
                }
                const double4 fr = sh.frame[lo];
                const double4 v = rec[sh.first[lo] + (f - sh.off[lo])];
                src = make_double4(fr.x + fr.w * v.x, fr.y + fr.w * v.y, fr.z + fr.w * v.z, v.w);
            }
            wave_sync();  // the previous tile has been read
            sh.tile[lane] = src;
            wave_sync();
            // the tile's sources (the last tile of a batch is partly filled)
            const int ns = (int)min(64u, total - f0);
            if (act) {
                if constexpr (F32) {
                    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, b0 = 0.0f, b1 = 0.0f, b2 = 0.0f, b3 = 0.0f;
#pragma unroll 4
                    for (int k = grp; k < ns; k += G) {
                        const double4 sk = sh.tile[k];
                        ad_pair32<true>(r0.x, r0.y, r0.z, sk, a0, a1, a2, a3);
                        ad_pair32<true>(r1.x, r1.y, r1.z, sk, b0, b1, b2, b3);
                    }
                    phi0 += (double)a0; ex0 += (double)a1; ey0 += (double)a2; ez0 += (double)a3;
                    phi1 += (double)b0; ex1 += (double)b1; ey1 += (double)b2; ez1 += (double)b3;
                } else {
#pragma unroll 4
                    for (int k = grp; k < ns; k += G) {
                        const double4 sk = sh.tile[k];
                        ad_pair<true>(r0.x, r0.y, r0.z, sk, phi0, ex0, ey0, ez0);
                        ad_pair<true>(r1.x, r1.y, r1.z, sk, phi1, ex1, ey1, ez1);
                    }
                }
            }
        }
    }
    // the groups' sums in group order, through LDS (tile and frame are free)
    wave_sync();
    sh.tile[lane] = make_double4(phi0, ex0, ey0, ez0);
    sh.frame[lane] = make_double4(phi1, ex1, ey1, ez1);
    wave_sync();
    if (grp == 0) {
        double4 a = sh.tile[slot], cc = sh.frame[slot];
        for (int k = 1; k < G; ++k) {
            const double4 x = sh.tile[k * T + slot], y = sh.frame[k * T + slot];
            a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
            cc.x += y.x; cc.y += y.y; cc.z += y.z; cc.w += y.w;
        }
        const double4 v0 = make_double4(a.x * s1, a.y * s2, a.z * s2, a.w * s2);
        const double4 v1 = make_double4(cc.x * s1, cc.y * s2, cc.z * s2, cc.w * s2);
        if constexpr (FUSE == 0) {
            if (live0) out[t0 + slot] = v0;
            if (live1) out[t0 + slot + T] = v1;
        } else {
            using To = std::conditional_t<FUSE == 2, double, float>;
            if (live0) combine_one<To>(c, t0 + slot, v0);
            if (live1) combine_one<To>(c, t0 + slot + T, v1);
        }
    }
}

template <int FUSE, bool F32>
__global__ __launch_bounds__(64 * kAdP2PWaves) void k_ad_p2p(
    const uint32_t *__restrict__ nunits, const int2 *__restrict__ units, const int *__restrict__ lbox,
    const uint32_t *__restrict__ lstart, const uint32_t *__restrict__ ou, const int *__restrict__ iu,
    const int *__restrict__ lev, const uint32_t *__restrict__ code, const uint32_t *__restrict__ ps,
    const uint32_t *__restrict__ pe, const double4 *__restrict__ rec, double4 *__restrict__ out, const Combine c) {
    __shared__ AdP2PShared shm[kAdP2PWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * kAdP2PWaves + wave;
    if (w >= (int64_t)*nunits) return;  // waves work alone: no block barrier below
    const int2 un = units[w];
    const int j = un.x;
    const int g = lbox[j];
    const uint32_t t0 = lstart[j] + (uint32_t)un.y, nt = min(64u, lstart[j + 1] - t0);
    ad_p2p_unit<FUSE, F32>(shm[wave], lane, g, lev[g], code[g], t0, nt, ou[g], ou[g + 1], iu, lev, code, ps, pe,
                           rec, out, c);
}

// Gathered M2L (FP64 MFMA), added to the locals: the targets of each (level,
// class) group, in tiles of 128 columns (4 waves x 2 x 16), against the K
// range of the class's 189 slots x S coefficients in chunks of 8; a column's
// source row for a slot comes from its V slots (an absent source reads the
// zero row).  A chunk's
// operator (R x 8, uniform over the block) is staged in LDS one chunk ahead;
// lane group q takes K index 4 j + q of a chunk (v_mfma_f64_16x16x4_f64).
template <int P>
__global__ __launch_bounds__(256) void k_ad_m2l(AdM2LPlan pl, const double *__restrict__ A,
                                                const int2 *__restrict__ cls, const double *__restrict__ M,
                                                const int *__restrict__ vidx, int64_t box2,
                                                const int *__restrict__ tgt, int64_t zero_row,
                                                double *__restrict__ Lc, double *__restrict__ partial) {
    constexpr int P2 = P * P, S = coef_stride(P), RT = m2l_rows(P) / 16, R = RT * 16;
    constexpr int NB = 2, KC = 8, ROWP = KC + 1, CPO = S / KC;
    constexpr int NEL = R * KC, EPT = (NEL + 255) / 256;
    constexpr int NCH = kOffsetsPerClass * CPO;
    __shared__ double As[2][R * ROWP];
    __shared__ int sA[kOffsetsPerClass];
    // block = part * units + tile: part takes chunks [kbeg, kend) of the K range
    const int64_t part = blockIdx.x / pl.units, b = blockIdx.x - part * pl.units;
    const int kbeg = (int)(part * NCH / pl.nsplit), kend = (int)((part + 1) * NCH / pl.nsplit);
    int gi = 0;
    for (int j = 1; j < pl.ngroups; ++j)
        if (b >= pl.grp[j].unit0) gi = j;
    const AdM2LGroup gr = pl.grp[gi];
    const int64_t tile = b - gr.unit0;
    const int k = gr.cls;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4, col = lane & 15;
    for (int i = tid; i < kOffsetsPerClass; i += 256) sA[i] = cls[k * kOffsetsPerClass + i].y * R * S;
    int64_t tbox[NB];
    const int *vrow[NB];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
        const int64_t c = tile * 128 + wave * NB * 16 + bb * 16 + col;
        tbox[bb] = c < gr.count ? tgt[gr.toff + c] : -1;
        vrow[bb] = tbox[bb] >= 0 ? vidx + (tbox[bb] - box2) * kOffsetsPerClass : nullptr;
    }
    __syncthreads();
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
    // source rows of the slot being fetched and of the next slot (its vidx
    // load is issued a slot ahead, so that no fetch waits on it); load_b is
    // called with a chunk index that never decreases and grows by at most one
    int srow[NB], snext[NB], pslot = kbeg / CPO;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
        srow[bb] = vrow[bb] ? vrow[bb][pslot] : -1;
        snext[bb] = (vrow[bb] && pslot + 1 < kOffsetsPerClass) ? vrow[bb][pslot + 1] : -1;
    }
    auto load_b = [&](int kc, double (&dst)[2][NB]) __attribute__((always_inline)) {
        const int slot = kc / CPO, c0 = KC * (kc - slot * CPO);
        if (slot != pslot) {
            pslot = slot;
#pragma unroll
            for (int bb = 0; bb < NB; ++bb) {
                srow[bb] = snext[bb];
                snext[bb] = (vrow[bb] && slot + 1 < kOffsetsPerClass) ? vrow[bb][slot + 1] : -1;
            }
        }
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            const double *src = M + (srow[bb] >= 0 ? (int64_t)srow[bb] : zero_row) * S + c0 + q;
#pragma unroll
            for (int j = 0; j < 2; ++j) dst[j][bb] = src[4 * j];
        }
    };
    f64x4 acc[RT][NB];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) acc[r][bb] = f64x4{0, 0, 0, 0};
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
        constexpr int ph = decltype(pc)::value;
        const double *as = As[ph];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const double av = as[(16 * r + col) * ROWP + 4 * j + q];
#pragma unroll
                for (int bb = 0; bb < NB; ++bb)
                    acc[r][bb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bc[j][bb], acc[r][bb], 0, 0, 0);
            }
        store_a(ph ^ 1, ar[ph]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int bb = 0; bb < NB; ++bb) bc[j][bb] = br[ph][j][bb];
        load_a(min(kc + 3, kend - 1), ar[ph]);
        load_b(min(kc + 3, kend - 1), br[ph]);
        __syncthreads();
    };
    int kc = kbeg;
    for (; kc + 1 < kend; kc += 2) {
        chunk(kc, std::integral_constant<int, 0>{});
        chunk(kc + 1, std::integral_constant<int, 1>{});
    }
    if (kc < kend) chunk(kc, std::integral_constant<int, 0>{});
    if (pl.nsplit == 1) {
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            if (tbox[bb] < 0) continue;
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * r + q + 4 * i;
                    if (row < P2) Lc[tbox[bb] * S + row] += acc[r][bb][i];
                }
        }
    } else {  // this part's sums of the tile's 128 columns, summed by k_ad_m2l_sum
        double *dst = partial + (part * pl.units + b) * 128 * P2;
#pragma unroll
        for (int bb = 0; bb < NB; ++bb)
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * r + q + 4 * i;
                    if (row < P2) dst[(wave * NB * 16 + bb * 16 + col) * P2 + row] = acc[r][bb][i];
                }
    }
}

// The K-split parts of the gathered M2L added into the locals in part order
// (one thread per (tile, column, row)).
__global__ void k_ad_m2l_sum(AdM2LPlan pl, int P2, int S, const int *__restrict__ tgt,
                             const double *__restrict__ partial, double *__restrict__ Lc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)128 * P2;
    if (i >= pl.units * per) return;
    const int64_t b = i / per;
    const int e = (int)(i - b * per), c = e / P2, row = e - c * P2;
    int gi = 0;
    for (int j = 1; j < pl.ngroups; ++j)
        if (b >= pl.grp[j].unit0) gi = j;
    const AdM2LGroup gr = pl.grp[gi];
    const int64_t t = (b - gr.unit0) * 128 + c;
    if (t >= gr.count) return;
    double v = 0.0;
    for (int k = 0; k < pl.nsplit; ++k) v += partial[((int64_t)k * pl.units + b) * per + e];
    Lc[(int64_t)tgt[gr.toff + t] * S + row] += v;
}

// Targets of levels >= 2 grouped by (level, class): block histograms in LDS
// and one global atomic per (block, group): counts (fill == NULL), or the
// fill, where each group's block range is reserved by that atomic and the
// LDS rank places the target in it (the order within a group does not
// change any result).
__global__ __launch_bounds__(256) void k_ad_class(int64_t box2, int64_t nb, const int *__restrict__ lev,
                                                  const uint32_t *__restrict__ code, unsigned int *__restrict__ cnt,
                                                  const int64_t *__restrict__ goff, unsigned int *__restrict__ fill,
                                                  int *__restrict__ tgt) {
    __shared__ unsigned int h[kAdMaxGroups], base[kAdMaxGroups];
    for (int k = threadIdx.x; k < kAdMaxGroups; k += 256) h[k] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int grp = -1;
    unsigned int rank = 0;
    if (i < nb) {
        const int64_t g = box2 + i;
        int64_t x, y, z;
        box_coords(code[g], x, y, z);
        grp = 8 * (lev[g] - 2) + (int)((x & 1) | ((y & 1) << 1) | ((z & 1) << 2));
        rank = atomicAdd(&h[grp], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kAdMaxGroups; k += 256)
        if (h[k]) base[k] = atomicAdd(fill ? fill + k : cnt + k, h[k]);
    __syncthreads();
    if (fill && grp >= 0) tgt[goff[grp] + base[grp] + rank] = (int)(box2 + i);
}

// ------------------------------------------------ M2L, binary16 encoding
// The mixed form's M2L on the adaptive tree: the uniform tree's binary16
// encoding (operators scaled per row and by the harmonic size of each
// column's degree, split hi + lo; multipoles scaled by the same column
// factors and by a power of two per level, split likewise; three products
// hi.hi + hi.lo + lo.hi on v_mfma_f32_16x16x32_f16, FP32 accumulation
// merged into FP64 every 256 K terms), with the multipole operand gathered
// through the V slots as in the FP64 kernel.

typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
// operator fragments as a native vector: a HIP uint4 is a struct, whose
// copies become memcpy calls that kept the prefetched fragments in scratch
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// Per-level maxima of |M_c rho_inv[c]|: one thread per (box, coefficient),
// an LDS maximum per level in the block, one global atomic per level and
// block (non-negative floats order like their bit patterns).
__global__ __launch_bounds__(256) void k_ad_level_max(int P, int64_t box2, int64_t nb, const int *__restrict__ lev,
                                                      const double *__restrict__ M, const float *__restrict__ rho_inv,
                                                      uint32_t *__restrict__ lmax) {
    __shared__ unsigned int lm[kLevelSlots];
    const int P2 = P * P, S = coef_stride(P);
    if (threadIdx.x < kLevelSlots) lm[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb * P2) {
        const int64_t g = box2 + i / P2;
        const int c = (int)(i % P2);
        const float v = (float)fabs(M[g * S + c]) * rho_inv[c];
        if (v > 0.0f) atomicMax(&lm[lev[g]], __float_as_uint(v));
    }
    __syncthreads();
    if (threadIdx.x < kLevelSlots && lm[threadIdx.x]) atomic_max_shared(lmax + threadIdx.x, lm[threadIdx.x]);
}

// One thread per 8-coefficient piece of rows box2 .. nbox (the last the zero
// row): scaled by rho_inv[c] 2^e(level) and split into binary16 hi and lo,
// stored hi8 then lo8 (32 bytes).
__global__ __launch_bounds__(256) void k_ad_pack_h(int P, int64_t box2, int64_t nbox, const int *__restrict__ lev,
                                                   const double *__restrict__ M, const float *__restrict__ rho_inv,
                                                   const uint32_t *__restrict__ lmax, uint4 *__restrict__ Bh) {
    const int S = coef_stride(P), PPO = S / 8;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (nbox + 1 - box2) * PPO) return;
    const int64_t g = box2 + i / PPO;
    const int pc = (int)(i % PPO);
    float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (g < nbox) {
        const float sc = ldexpf(1.0f, level_scale_exp(lmax[lev[g]]));
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = 8 * pc + k;
            const float r = rho_inv[c];  // 0 past p^2 (padding, never written)
            v[k] = r != 0.0f ? (float)M[g * S + c] * (r * sc) : 0.0f;
        }
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
    Bh[2 * (g * PPO + pc)] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    Bh[2 * (g * PPO + pc) + 1] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
}

// Tiles of 128 targets of one (level, class) group, 4 waves x 2 blocks of 16
// columns; K in steps of 32 (4 pieces of 8; lane group q takes piece
// 4 kc + q, which belongs to slot (4 kc + q) / (S/8) of the class).  A step's
// operator fragments (2 parts x RT row tiles, 1 KB each) are copied into LDS
// one step ahead through registers; each lane's multipole fragments come
// from the row its column's V slot names (the zero row when absent), the
// slot table read a slot ahead and the fragments three steps ahead.
template <int P>
__global__ __launch_bounds__(256) void k_ad_m2l_h(AdM2LPlan pl, const uint16_t *__restrict__ Ah, size_t astride,
                                                  const int2 *__restrict__ cls, const uint4 *__restrict__ Bh,
                                                  const int *__restrict__ vidx, int64_t box2,
                                                  const int *__restrict__ tgt, int64_t zero_row,
                                                  const uint32_t *__restrict__ lmax,
                                                  const float *__restrict__ oscale, double *__restrict__ Lc,
                                                  double *__restrict__ partial) {
    constexpr int P2 = P * P, S = coef_stride(P), PPO = S / 8, RT = m2l_rows(P) / 16, R = RT * 16, NB = 2;
    constexpr int NPC = kOffsetsPerClass * PPO;  // pieces of a class
    constexpr int NCH = (NPC + 3) / 4;           // K steps
    constexpr int NFR = 2 * RT;                  // operator fragments per step
    constexpr int EPT = (NFR * 64 + 255) / 256;  // of them per thread
    constexpr int D = 3;                         // multipole steps in flight
    __shared__ u32x4_t As[2][NFR * 64];
    __shared__ int sA[kOffsetsPerClass + 1];
    const int64_t part = blockIdx.x / pl.units, b = blockIdx.x - part * pl.units;
    const int kbeg = (int)(part * NCH / pl.nsplit), kend = (int)((part + 1) * NCH / pl.nsplit);
    int gi = 0;
    for (int j = 1; j < pl.ngroups; ++j)
        if (b >= pl.grp[j].unit0) gi = j;
    const AdM2LGroup gr = pl.grp[gi];
    const int64_t tile = b - gr.unit0;
    const int k = gr.cls;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4, col = lane & 15;
    for (int i = tid; i <= kOffsetsPerClass; i += 256)
        sA[i] = (i < kOffsetsPerClass ? cls[k * kOffsetsPerClass + i].y : kNumOffsets) * R * S;
    int64_t tbox[NB];
    const int *vrow[NB];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
        const int64_t c = tile * 128 + wave * NB * 16 + bb * 16 + col;
        tbox[bb] = c < gr.count ? tgt[gr.toff + c] : -1;
        vrow[bb] = tbox[bb] >= 0 ? vidx + (tbox[bb] - box2) * kOffsetsPerClass : nullptr;
    }
    __syncthreads();
    auto load_a = [&](int kc, u32x4_t (&dst)[EPT]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + 256 * i;
            if (NFR * 64 % 256 == 0 || e < NFR * 64) {
                const int fr = e >> 6, L = e & 63, sp = fr / RT, r = fr - sp * RT;
                const int g = 4 * kc + (L >> 4);
                const int slot = g < NPC ? g / PPO : kOffsetsPerClass, pc = g < NPC ? g - (g / PPO) * PPO : 0;
                dst[i] = *(const u32x4_t *)(Ah + sp * astride + sA[slot] + (r * PPO + pc) * 128 + (L & 15) * 8);
            }
        }
    };
    auto store_a = [&](int buf, const u32x4_t (&src)[EPT]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + 256 * i;
            if (NFR * 64 % 256 == 0 || e < NFR * 64) As[buf][e] = src[i];
        }
    };
    // this lane's source rows: srow for the slot of the piece being fetched,
    // snext for the slot after it (loaded a slot ahead when a slot spans at
    // least one step, else read when needed)
    int pslot = -2, srow[NB], snext[NB];  // -2: no slot fetched yet
    auto row_of = [&](int bb, int slot) __attribute__((always_inline)) -> int {
        return (vrow[bb] && slot < kOffsetsPerClass) ? vrow[bb][slot] : -1;
    };
    auto load_b = [&](int kc, uint4 (&hi)[NB], uint4 (&lo)[NB]) __attribute__((always_inline)) {
        const int g = 4 * kc + q;
        const int slot = g < NPC ? g / PPO : kOffsetsPerClass, pc = g < NPC ? g - (g / PPO) * PPO : 0;
        if (slot != pslot) {
            if constexpr (PPO >= 4) {
                if (slot == pslot + 1) {
#pragma unroll
                    for (int bb = 0; bb < NB; ++bb) {
                        srow[bb] = snext[bb];
                        snext[bb] = row_of(bb, slot + 1);
                    }
                } else {
#pragma unroll
                    for (int bb = 0; bb < NB; ++bb) {
                        srow[bb] = row_of(bb, slot);
                        snext[bb] = row_of(bb, slot + 1);
                    }
                }
            } else {
#pragma unroll
                for (int bb = 0; bb < NB; ++bb) srow[bb] = row_of(bb, slot);
            }
            pslot = slot;
        }
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            const uint4 *src = Bh + 2 * ((srow[bb] >= 0 ? (int64_t)srow[bb] : zero_row) * PPO + pc);
            hi[bb] = src[0];
            lo[bb] = src[1];
        }
    };
    f32x4_t acc[RT][NB];
    f64x4 acc64[RT][NB];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            acc[r][bb] = f32x4_t{0, 0, 0, 0};
            acc64[r][bb] = f64x4{0, 0, 0, 0};
        }
    u32x4_t ar[EPT];
    uint4 bhi[D][NB], blo[D][NB];
    load_a(kbeg, ar);
    store_a(0, ar);
#pragma unroll
    for (int d = 0; d < D; ++d) load_b(min(kbeg + d, kend - 1), bhi[d], blo[d]);
    load_a(min(kbeg + 1, kend - 1), ar);
    __syncthreads();
    auto step = [&](int kc, auto dc) __attribute__((always_inline)) {
        constexpr int d = decltype(dc)::value % D, ph = decltype(dc)::value & 1;
        const u32x4_t *as = As[ph];
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const f16x8_t ah = __builtin_bit_cast(f16x8_t, as[r * 64 + lane]);
            const f16x8_t al = __builtin_bit_cast(f16x8_t, as[(RT + r) * 64 + lane]);
#pragma unroll
            for (int bb = 0; bb < NB; ++bb) {
                const f16x8_t bh = __builtin_bit_cast(f16x8_t, bhi[d][bb]);
                const f16x8_t bl = __builtin_bit_cast(f16x8_t, blo[d][bb]);
                acc[r][bb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, acc[r][bb], 0, 0, 0);
                acc[r][bb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, acc[r][bb], 0, 0, 0);
                acc[r][bb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, acc[r][bb], 0, 0, 0);
            }
        }
        store_a(ph ^ 1, ar);  // step kc + 1, read by every wave after the barrier below
        load_a(min(kc + 2, kend - 1), ar);
        load_b(min(kc + D, kend - 1), bhi[d], blo[d]);
        __syncthreads();
    };
    auto merge = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int bb = 0; bb < NB; ++bb) {
#pragma unroll
                for (int i = 0; i < 4; ++i) acc64[r][bb][i] += (double)acc[r][bb][i];
                acc[r][bb] = f32x4_t{0, 0, 0, 0};
            }
    };
    // six steps per pass keep both the LDS parity and the multipole ring
    // position compile-time constants; merges every 6 steps (192 K terms)
    int kc = kbeg;
    for (; kc + 5 < kend; kc += 6) {
        step(kc, std::integral_constant<int, 0>{});
        step(kc + 1, std::integral_constant<int, 1>{});
        step(kc + 2, std::integral_constant<int, 2>{});
        step(kc + 3, std::integral_constant<int, 3>{});
        step(kc + 4, std::integral_constant<int, 4>{});
        step(kc + 5, std::integral_constant<int, 5>{});
        merge();
    }
    // the remaining steps, with the ring positions they would have had
    if (kc < kend) step(kc, std::integral_constant<int, 0>{});
    if (kc + 1 < kend) step(kc + 1, std::integral_constant<int, 1>{});
    if (kc + 2 < kend) step(kc + 2, std::integral_constant<int, 2>{});
    if (kc + 3 < kend) step(kc + 3, std::integral_constant<int, 3>{});
    if (kc + 4 < kend) step(kc + 4, std::integral_constant<int, 4>{});
    merge();
    // undo the encoding: row r carries the table's row scale and the level's
    // operand scale (powers of two)
    const int sh = -level_scale_exp(lmax[gr.lev]);
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * r + 4 * q + i;
            const double f = row < P2 ? ldexp((double)oscale[row], sh) : 0.0;
#pragma unroll
            for (int bb = 0; bb < NB; ++bb) acc64[r][bb][i] *= f;
        }
    if (pl.nsplit == 1) {
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
            if (tbox[bb] < 0) continue;
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * r + 4 * q + i;
                    if (row < P2) Lc[tbox[bb] * S + row] += acc64[r][bb][i];
                }
        }
    } else {  // this part's sums of the tile's 128 columns, summed by k_ad_m2l_sum
        double *dst = partial + (part * pl.units + b) * 128 * P2;
#pragma unroll
        for (int bb = 0; bb < NB; ++bb)
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * r + 4 * q + i;
                    if (row < P2) dst[(wave * NB * 16 + bb * 16 + col) * P2 + row] = acc64[r][bb][i];
                }
    }
}

// ---------------------------------------------------------- host helpers
static inline unsigned ad_blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t ad_launch_root(uint32_t n, uint32_t *code, uint32_t *ps, uint32_t *pe, int *parent, hipStream_t st) {
    k_ad_root<<<1, 1, 0, st>>>(n, code, ps, pe, parent);
    return hipGetLastError();
}

hipError_t ad_launch_count(int64_t b0, int64_t nb, int l, int Lf, int leaf_max, const uint32_t *code,
                           const uint32_t *ps, const uint32_t *pe, const KeyIndex &ki, uint8_t *leaf,
                           uint32_t *nchild, uint8_t *cmask, hipStream_t st) {
    k_ad_count<<<ad_blocks(nb, 256), 256, 0, st>>>(b0, nb, l, Lf, leaf_max, code, ps, pe, ki, leaf, nchild, cmask);
    return hipGetLastError();
}

hipError_t ad_launch_children(int64_t b0, int64_t nb, int l, int Lf, int64_t next0, const KeyIndex &ki,
                              const uint32_t *coff, const uint8_t *cmask, uint32_t *code, uint32_t *ps,
                              uint32_t *pe, int *parent, int *child, hipStream_t st) {
    k_ad_children<<<ad_blocks(nb, 256), 256, 0, st>>>(b0, nb, l, Lf, next0, ki, coff, cmask, code, ps, pe, parent,
                                                       child);
    return hipGetLastError();
}

hipError_t ad_launch_structure(int64_t nbox, int nlev, const int64_t *off_host, const int64_t *off_dev,
                               const uint32_t *code, const int *parent, const int *child, int *lev, int *col,
                               const int2 *cls, int *vidx, hipStream_t st) {
    k_ad_levels<<<ad_blocks(nbox, 256), 256, 0, st>>>(nbox, off_dev, nlev, lev);
    for (int l = 0; l < nlev; ++l) {
        const int64_t nb = off_host[l + 1] - off_host[l];
        if (nb > 0) k_ad_colleagues<<<ad_blocks(27 * nb, 256), 256, 0, st>>>(off_host[l], nb, l, code, col);
    }
    for (int l = 2; l < nlev; ++l) {
        const int64_t nb = off_host[l + 1] - off_host[l];
        if (nb > 0)
            k_ad_vslots<<<ad_blocks(kOffsetsPerClass * nb, 256), 256, 0, st>>>(off_host[l], nb, code, parent, col,
                                                                                child, cls,
                                                             vidx + 189 * (off_host[l] - off_host[2]));
    }
    return hipGetLastError();
}

hipError_t ad_launch_lists(int64_t nbox, int pass, const int *lev, const uint32_t *code, const int *parent,
                           const int *col, const int *child, const uint8_t *leaf, uint32_t *nu, uint32_t *nw,
                           uint32_t *nx, const uint32_t *ou, const uint32_t *ow, const uint32_t *ox, int *iu,
                           int *iw, int *ix, hipStream_t st) {
    k_ad_lists<<<ad_blocks(27 * nbox, 128), 128, 0, st>>>(nbox, pass, lev, code, parent, col, child, leaf, nu, nw, nx,
                                                      ou, ow, ox, iu, iw, ix);
    return hipGetLastError();
}

hipError_t ad_launch_box_offsets(int64_t nbox, const uint32_t *s27, uint32_t *ou, uint32_t *ow, uint32_t *ox,
                                 hipStream_t st) {
    k_ad_box_offsets<<<ad_blocks(nbox + 1, 256), 256, 0, st>>>(nbox, s27, ou, ow, ox);
    return hipGetLastError();
}

hipError_t ad_launch_heads(int64_t nbox, const uint8_t *leaf, const uint32_t *ps, const uint32_t *pe,
                           uint32_t *is_head, int *head, hipStream_t st) {
    k_ad_heads<<<ad_blocks(nbox, 256), 256, 0, st>>>(nbox, leaf, ps, pe, is_head, head);
    return hipGetLastError();
}

hipError_t ad_launch_leaflist(int64_t n, int64_t nleaf, const uint32_t *is_head, const uint32_t *hoff,
                              const int *head, const uint32_t *ps, int *lbox, uint32_t *lstart, uint8_t *llev,
                              const int *lev, unsigned int *mx, hipStream_t st) {
    k_ad_leaflist<<<ad_blocks(n, 256), 256, 0, st>>>(n, is_head, hoff, head, ps, lbox, lstart, llev, lev);
    k_ad_leafmax<<<(unsigned)std::min<int64_t>(256, (nleaf + 255) / 256), 256, 0, st>>>(nleaf, lstart, mx);
    return hipGetLastError();
}

hipError_t ad_launch_counts(int64_t nbox, int64_t box2, const uint8_t *leaf, const uint32_t *ps, const uint32_t *pe,
                            const uint32_t *ou, const int *iu, const uint32_t *ow, const uint32_t *ox, const int *ix,
                            const int *vidx, unsigned long long *out, hipStream_t st) {
    k_ad_counts<<<ad_blocks(nbox, 256), 256, 0, st>>>(nbox, box2, leaf, ps, pe, ou, iu, ow, ox, ix, vidx, out);
    return hipGetLastError();
}

hipError_t ad_launch_records(int64_t n, int dtype, const uint32_t *hoff, const int *lbox, const int *lev,
                             const uint32_t *code, const uint32_t *perm, const void *pos, const double lo[3],
                             double size, double4 *rec, hipStream_t st) {
    if (dtype == FMM_F64)
        k_ad_records<double><<<ad_blocks(n, 256), 256, 0, st>>>(n, hoff, lbox, lev, code, perm, (const double *)pos,
                                                                lo[0], lo[1], lo[2], 1.0 / size, rec);
    else
        k_ad_records<float><<<ad_blocks(n, 256), 256, 0, st>>>(n, hoff, lbox, lev, code, perm, (const float *)pos,
                                                               lo[0], lo[1], lo[2], 1.0 / size, rec);
    return hipGetLastError();
}

#define AD_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t ad_launch_p2m(int P, int64_t nleaf, const int *lbox, const uint32_t *lstart, const uint8_t *llev, int adj,
                         const double4 *rec, double *M, bool f32, hipStream_t st) {
    if (nleaf == 0) return hipSuccess;
    switch (P) {
#define X(PP)                                                                                                   \
    case PP:                                                                                                    \
        if (f32) k_ad_p2m<PP, float><<<(unsigned)nleaf, 64, 0, st>>>(lbox, lstart, llev, adj, rec, M);         \
        else k_ad_p2m<PP, double><<<(unsigned)nleaf, 64, 0, st>>>(lbox, lstart, llev, adj, rec, M);            \
        break;
        AD_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// boxes per block of k_ad_m2m (its BX)
static constexpr int m2m_boxes(int P) {
    return 4096 / (8 * P * P) < 1 ? 1 : (4096 / (8 * P * P) > 8 ? 8 : 4096 / (8 * P * P));
}

hipError_t ad_launch_m2m(int P, int64_t b0, int64_t nb, const uint8_t *leaf, const int *child, const double *tab,
                         double *M, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    switch (P) {
#define X(PP)                                                                                                   \
    case PP:                                                                                                    \
        k_ad_m2m<PP><<<(unsigned)((nb + m2m_boxes(PP) - 1) / m2m_boxes(PP)), 256, 0, st>>>(b0, nb, leaf, child,  \
                                                                                         tab, M);                \
        break;
        AD_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t ad_launch_l2l(int P, int64_t b0, int64_t nb, const uint32_t *code, const int *parent, const double *tab,
                         double *Lc, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    switch (P) {
#define X(PP) case PP: k_ad_l2l<PP><<<(unsigned)nb, 256, 0, st>>>(b0, code, parent, tab, Lc); break;
        AD_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t ad_launch_m2l(int P, const AdM2LPlan &pl, const double *A, const int2 *cls, const double *M,
                         const int *vidx, int64_t box2, const int *tgt, int64_t zero_row, double *Lc, double *partial,
                         hipStream_t st) {
    if (pl.units == 0) return hipSuccess;
    if (pl.nsplit < 1 || (pl.nsplit > 1 && !partial)) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)(pl.units * pl.nsplit);
    switch (P) {
#define X(PP) \
    case PP: k_ad_m2l<PP><<<nb, 256, 0, st>>>(pl, A, cls, M, vidx, box2, tgt, zero_row, Lc, partial); break;
        AD_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    if (pl.nsplit > 1)
        k_ad_m2l_sum<<<ad_blocks(pl.units * 128 * P * P, 256), 256, 0, st>>>(pl, P * P, coef_stride(P), tgt, partial,
                                                                             Lc);
    return hipGetLastError();
}

hipError_t ad_launch_pack_h(int P, int64_t box2, int64_t nbox, const int *lev, const double *M,
                            const float *rho_inv, uint32_t *lmax, void *Bh, hipStream_t st) {
    const int64_t nb = nbox - box2;
    if (nb > 0)
        k_ad_level_max<<<ad_blocks(nb * P * P, 256), 256, 0, st>>>(P, box2, nb, lev, M, rho_inv, lmax);
    k_ad_pack_h<<<ad_blocks((nb + 1) * (coef_stride(P) / 8), 256), 256, 0, st>>>(P, box2, nbox, lev, M, rho_inv,
                                                                                 lmax, (uint4 *)Bh);
    return hipGetLastError();
}

hipError_t ad_launch_m2l_h(int P, const AdM2LPlan &pl, const uint16_t *Ah, size_t astride, const int2 *cls,
                           const void *Bh, const int *vidx, int64_t box2, const int *tgt, int64_t zero_row,
                           const uint32_t *lmax, const float *oscale, double *Lc, double *partial, hipStream_t st) {
    if (pl.units == 0) return hipSuccess;
    if (pl.nsplit < 1 || (pl.nsplit > 1 && !partial)) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)(pl.units * pl.nsplit);
    switch (P) {
#define X(PP)                                                                                             \
    case PP:                                                                                              \
        k_ad_m2l_h<PP><<<nb, 256, 0, st>>>(pl, Ah, astride, cls, (const uint4 *)Bh, vidx, box2, tgt, zero_row, \
                                           lmax, oscale, Lc, partial);                                     \
        break;
        AD_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    if (pl.nsplit > 1)
        k_ad_m2l_sum<<<ad_blocks(pl.units * 128 * P * P, 256), 256, 0, st>>>(pl, P * P, coef_stride(P), tgt, partial,
                                                                             Lc);
    return hipGetLastError();
}

hipError_t ad_launch_class(int64_t box2, int64_t nb, const int *lev, const uint32_t *code, unsigned int *cnt,
                           const int64_t *goff, unsigned int *fill, int *tgt, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    k_ad_class<<<ad_blocks(nb, 256), 256, 0, st>>>(box2, nb, lev, code, cnt, goff, fill, tgt);
    return hipGetLastError();
}

hipError_t ad_launch_p2l(int P, int64_t nbox, const uint32_t *ox, const int *ix, const int *lev,
                         const uint32_t *code, const uint32_t *ps, const uint32_t *pe, int adj, const double4 *rec,
                         double *Lc, bool f32, hipStream_t st) {
    switch (P) {
#define X(PP)                                                                                                   \
    case PP:                                                                                                    \
        if (f32) k_ad_p2l<PP, float><<<(unsigned)nbox, 64, 0, st>>>(ox, ix, lev, code, ps, pe, adj, rec, Lc);  \
        else k_ad_p2l<PP, double><<<(unsigned)nbox, 64, 0, st>>>(ox, ix, lev, code, ps, pe, adj, rec, Lc);     \
        break;
        AD_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t ad_launch_l2p(int P, int64_t nleaf, const int *lbox, const uint32_t *lstart, const uint8_t *llev,
                         int adj, const double4 *rec, const double *Lc, double4 *out, bool f32, hipStream_t st) {
    switch (P) {
#define X(PP)                                                                                                   \
    case PP:                                                                                                    \
        if (f32) k_ad_l2p<PP, float><<<(unsigned)nleaf, 64, 0, st>>>(lbox, lstart, llev, adj, rec, Lc, out);   \
        else k_ad_l2p<PP, double><<<(unsigned)nleaf, 64, 0, st>>>(lbox, lstart, llev, adj, rec, Lc, out);      \
        break;
        AD_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t ad_launch_m2p(int P, int64_t max_units, const uint32_t *nunits, const int2 *units, int adj,
                         const int *lbox, const uint32_t *lstart, const uint32_t *ow, const int *iw, const int *lev,
                         const uint32_t *code, const double4 *rec, const double *M, double4 *out, bool f32,
                         hipStream_t st) {
    switch (P) {
#define X(PP)                                                                                                   \
    case PP:                                                                                                    \
        if (f32)                                                                                                \
            k_ad_m2p<PP, float><<<(unsigned)max_units, 64, 0, st>>>(nunits, units, adj, lbox, lstart, ow, iw,   \
                                                                    lev, code, rec, M, out);                    \
        else                                                                                                    \
            k_ad_m2p<PP, double><<<(unsigned)max_units, 64, 0, st>>>(nunits, units, adj, lbox, lstart, ow, iw,  \
                                                                     lev, code, rec, M, out);                   \
        break;
        AD_CASES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t ad_launch_units(int64_t nleaf, int pass, const uint32_t *lstart, const int *lbox, const uint32_t *ou,
                           const uint32_t *ow, const int *iu, const uint32_t *ps, const uint32_t *pe, uint32_t *cnt,
                           const uint32_t *uoff, int2 *units, int2 *units_m, hipStream_t st) {
    k_ad_units<<<ad_blocks(nleaf, 256), 256, 0, st>>>(nleaf, pass, lstart, lbox, ou, ow, iu, ps, pe, cnt, uoff, units,
                                                      units_m);
    return hipGetLastError();
}

hipError_t ad_launch_p2p(int64_t max_units, const uint32_t *nunits, const int2 *units, const int *lbox,
                         const uint32_t *lstart, const uint32_t *ou, const int *iu, const int *lev, const uint32_t *code,
                         const uint32_t *ps, const uint32_t *pe, const double4 *rec, double4 *out, const Combine *fuse,
                         bool f32, hipStream_t st) {
    const Combine c = fuse ? *fuse : Combine{};
    const unsigned grid = ad_blocks(max_units, kAdP2PWaves);
#define AD_P2P(FU, F)                                                                                          \
    k_ad_p2p<FU, F><<<grid, 64 * kAdP2PWaves, 0, st>>>(nunits, units, lbox, lstart, ou, iu, lev, code, ps, pe, \
                                                        rec, out, c)
    const int fu = !fuse ? 0 : fuse->dtype == FMM_F64 ? 2 : 1;
    if (f32) {
        if (fu == 0) AD_P2P(0, true);
        else if (fu == 2) AD_P2P(2, true);
        else AD_P2P(1, true);
    } else {
        if (fu == 0) AD_P2P(0, false);
        else if (fu == 2) AD_P2P(2, false);
        else AD_P2P(1, false);
    }
#undef AD_P2P
    return hipGetLastError();
}

}  // namespace fmm

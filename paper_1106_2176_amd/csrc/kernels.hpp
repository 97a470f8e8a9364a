// kernels.hpp -- launchers of the device kernels (all asynchronous on `st`).
#pragma once
#include <algorithm>

#include "common.hpp"

namespace fmm {

// tree.hip
// keys + leaf counts + ranks at `level` (zeroes cnt and counters[0..1] first);
// with cnt NULL the keys alone
hipError_t launch_keys(int64_t n, int dtype, const void *pos, const double lo[3], double size,
                       int level, uint32_t *key10, uint32_t *cnt, uint32_t *rank,
                       unsigned int *counters, hipStream_t st);
// leaf counts + ranks at another level from the keys (counters[1] restarts)
hipError_t launch_hist(int64_t n, const uint32_t *key10, int level, uint32_t *cnt, uint32_t *rank,
                       unsigned int *counters, hipStream_t st);
// zero `words` 32-bit words with a kernel (not a memset node when captured)
hipError_t launch_zero(uint32_t *p, int64_t words, hipStream_t st);
int64_t scan_scratch_words(int64_t nb);
hipError_t launch_scan(int64_t nb, const uint32_t *in, uint32_t *out, uint32_t *scratch,
                       hipStream_t st);
// exclusive scan (out[0..nb], total at out[nb]) and the maximum count into
// *mx (one kernel up to 32768 counts; *mx must be zero before a larger scan).
// With host (device-visible pinned words) the one-kernel form also stores
// *nbad and the maximum there and sets *host_done; the caller copies them
// otherwise.
hipError_t launch_scan_max(int64_t nb, const uint32_t *in, uint32_t *out, uint32_t *scratch,
                           unsigned int *mx, const unsigned int *nbad, unsigned int *host, bool *host_done,
                           hipStream_t st);
hipError_t launch_sort(int64_t n, int level, uint32_t skip, const uint32_t *key10, const uint32_t *rank,
                       const uint32_t *start, uint32_t *tmp, int dtype, const void *pos,
                       const double lo[3], double size, uint32_t *perm, int4 *xyz32,
                       double4 *xyz64, hipStream_t st);
// Key sort of an adaptive build (no bin per key of the finest level):
// stable radix sort by the key at `level`, perm (sorted position -> input
// index) and the sorted keys skey.  Scratch: keys_a, keys_b and vals of n
// words, hist of key_sort_hist_words(n), off of one more, scan of
// scan_scratch_words(key_sort_hist_words(n)).
struct KeySortWork {
    uint32_t *keys_a, *keys_b, *vals, *hist, *off, *scan;
};
int64_t key_sort_hist_words(int64_t n);
hipError_t launch_key_sort(int64_t n, int level, const uint32_t *key10, const KeySortWork &w, uint32_t *perm,
                           uint32_t *skey, hipStream_t st);
// FP64 leaf-relative records at `level` in sorted order
hipError_t launch_records(int64_t n, int level, const uint32_t *perm, const uint32_t *key10, int dtype,
                          const void *pos, const double lo[3], double size, double4 *xyz64, hipStream_t st);
// cstart[x], x in [0, 8^cl]: the first sorted position whose key at level
// cl is >= x, from the keys at `level` >= cl sorted (skey)
hipError_t launch_key_starts(int64_t n, int level, int cl, const uint32_t *skey, uint32_t *cstart, hipStream_t st);
hipError_t launch_pair_count(int level, const uint32_t *start, unsigned long long *out,
                             hipStream_t st);

// p2p.hip
// with fuse non-NULL the kernel ends with the combine (no near partials)
hipError_t launch_p2p(int L, bool f64, const void *src, const uint32_t *start, double4 *out, const Combine *fuse,
                      hipStream_t st);

// far.hip
// P2M at the leaves; with perm non-NULL it first stores each particle's
// charge q[perm[i]] (caller dtype q_dtype) into its sorted record i
// clear (optional): the kLevelSlots per-level maxima of the binary16 M2L
// encoding, zeroed by P2M's first block
hipError_t launch_p2m(int P, int L, bool f64, void *src, const uint32_t *start, void *M,
                      double scale, const uint32_t *perm, const void *q, int q_dtype,
                      uint32_t *clear, hipStream_t st);
// with fuse non-NULL (fuse->farf = the near partials) it ends with the combine
hipError_t launch_l2p(int P, int L, bool f64, const void *src, const uint32_t *start,
                      const void *Lc, double4 *out, const Combine *fuse, hipStream_t st);
hipError_t launch_transfer(bool up, int P, int lp, int in_f64, int out_f64, const void *in,
                           void *out, const void *tab32, const void *tab64, hipStream_t st);
// M2L operand grids of levels 2..L in one launch; level i of the plan:
// multipoles in[i] (FP64 when in_f64[i]) -> padded grid out[i] (FP64 when
// f64_out, else FP32, or with lmax the binary16 parts of the scaled
// multipoles); row0 = first padded row of each level, row0[nlev] = all rows.
// With lmax (kLevelSlots words, indexed by level, cleared beforehand) a
// first kernel takes each level's largest |M_c rho_inv[c]|, from which the
// level's power-of-two scale follows (level_scale_exp).
constexpr int kMaxPackLev = FMM_MAX_LEVEL;
struct PackPlan {
    int nlev;
    int level[kMaxPackLev];
    int in_f64[kMaxPackLev];
    int64_t row0[kMaxPackLev + 1];
    int64_t blk0[kMaxPackLev + 1];  // filled by launch_pack
    const void *in[kMaxPackLev];
    void *out[kMaxPackLev];
    uint32_t *lmax;                 // NULL: FP32 / FP64 grids
    const float *rho_inv;           // [S]: 1 / rho of each coefficient's degree
};
hipError_t launch_pack(int P, bool f64_out, const PackPlan &pl, hipStream_t st);
hipError_t launch_gather_q(int64_t n, int dtype, bool f64, const uint32_t *perm, const void *q,
                           void *xyzq, hipStream_t st);
hipError_t launch_combine(int64_t n, const double4 *nearf, const Combine &c, hipStream_t st);
hipError_t launch_combine_grad(int64_t n, int dtype, const uint32_t *perm, const double4 *nearf,
                               const double4 *farf, double inv_w, const void *q, const void *w,
                               const void *Eq, void *gq, void *gx, hipStream_t st);

// Rotation-based M2L tables (FP64 form), compact per offset id: D by degree
// blocks, (2n+1)^2 each, the block of degree n first at rot_deg_off(n); Tz by
// (order m, kind) blocks of (p-m)^2, m = 0 cosine only, then the cosine and
// sine blocks of m = 1, 2, ..., row = output degree - m, column = input
// degree - m.
__host__ __device__ constexpr int rot_deg_off(int n) { return n * (4 * n * n - 1) / 3; }
__host__ __device__ constexpr int rot_size(int P) { return rot_deg_off(P); }
__host__ __device__ constexpr int tz_off(int P, int m, int kind) {
    int o = 0;
    for (int j = 0; j < m; ++j) o += (j == 0 ? 1 : 2) * (P - j) * (P - j);
    return o + (kind ? (P - m) * (P - m) : 0);
}
__host__ __device__ constexpr int tz_size(int P) { return tz_off(P, P, 0); }
// every level 2..L in one launch, B[l] = FP64 padded grid, Lc[l] FP64 output
hipError_t launch_m2l_rot(int P, int L, void *const *B, void *const *Lc, const double *rot,
                          const double *tz, const int2 *cls, hipStream_t st);

// adaptive.hip: the adaptive octree (FP64 form); see the file's header for
// the layout.  Build steps (per level, host-driven) and list construction:
hipError_t ad_launch_root(uint32_t n, uint32_t *code, uint32_t *ps, uint32_t *pe, int *parent, hipStream_t st);
// the sorted keys of the finest level Lf and the first position of each
// key of level cl <= Lf (cstart[8^cl + 1]), for the box ranges
struct KeyIndex {
    const uint32_t *cstart, *skey;
    int Lf, cl;
};
hipError_t ad_launch_count(int64_t b0, int64_t nb, int l, int Lf, int leaf_max, const uint32_t *code,
                           const uint32_t *ps, const uint32_t *pe, const KeyIndex &ki, uint8_t *leaf,
                           uint32_t *nchild, uint8_t *cmask, hipStream_t st);
hipError_t ad_launch_children(int64_t b0, int64_t nb, int l, int Lf, int64_t next0, const KeyIndex &ki,
                              const uint32_t *coff, const uint8_t *cmask, uint32_t *code, uint32_t *ps,
                              uint32_t *pe, int *parent, int *child, hipStream_t st);
hipError_t ad_launch_structure(int64_t nbox, int nlev, const int64_t *off_host, const int64_t *off_dev,
                               const uint32_t *code, const int *parent, const int *child, int *lev, int *col,
                               const int2 *cls, int *vidx, hipStream_t st);
// one thread per (box, direction): pass 0 counts [27 nbox] each, pass 1
// fills at the scanned per-(box, direction) offsets
hipError_t ad_launch_lists(int64_t nbox, int pass, const int *lev, const uint32_t *code, const int *parent,
                           const int *col, const int *child, const uint8_t *leaf, uint32_t *nu, uint32_t *nw,
                           uint32_t *nx, const uint32_t *ou, const uint32_t *ow, const uint32_t *ox, int *iu,
                           int *iw, int *ix, hipStream_t st);
// per-box list offsets ou/ow/ox [nbox + 1] from the three per-(box,
// direction) scans stored one after another, each 27 nbox + 1 long
hipError_t ad_launch_box_offsets(int64_t nbox, const uint32_t *s27, uint32_t *ou, uint32_t *ow, uint32_t *ox,
                                 hipStream_t st);
hipError_t ad_launch_heads(int64_t nbox, const uint8_t *leaf, const uint32_t *ps, const uint32_t *pe,
                           uint32_t *is_head, int *head, hipStream_t st);
// leaves in particle order, and the fullest leaf's count into *mx
hipError_t ad_launch_leaflist(int64_t n, int64_t nleaf, const uint32_t *is_head, const uint32_t *hoff,
                              const int *head, const uint32_t *ps, int *lbox, uint32_t *lstart, uint8_t *llev,
                              const int *lev, unsigned int *mx, hipStream_t st);
// out[4] (zeroed): ordered P2P pairs incl. self, V entries, W and X (particle, box) pairs
hipError_t ad_launch_counts(int64_t nbox, int64_t box2, const uint8_t *leaf, const uint32_t *ps, const uint32_t *pe,
                            const uint32_t *ou, const int *iu, const uint32_t *ow, const uint32_t *ox, const int *ix,
                            const int *vidx, unsigned long long *out, hipStream_t st);
hipError_t ad_launch_records(int64_t n, int dtype, const uint32_t *hoff, const int *lbox, const int *lev,
                             const uint32_t *code, const uint32_t *perm, const void *pos, const double lo[3],
                             double size, double4 *rec, hipStream_t st);
hipError_t ad_launch_class(int64_t box2, int64_t nb, const int *lev, const uint32_t *code, unsigned int *cnt,
                           const int64_t *goff, unsigned int *fill, int *tgt, hipStream_t st);
// M2L targets: groups (level >= 2, class) of the target list, tiles of 128
struct AdM2LGroup {
    int64_t unit0;  // first block of the group
    int64_t toff;   // first target of the group in the target list
    int64_t count;  // targets in the group
    int cls;        // child class of the group's targets
    int lev;        // level of the group's targets
};
constexpr int kAdMaxGroups = 8 * (FMM_MAX_LEVEL - 1);
struct AdM2LPlan {
    int ngroups;
    int nsplit;      // K-split parts (1: the blocks add straight into the locals)
    int64_t units;   // tiles of 128 targets over all groups
    AdM2LGroup grp[kAdMaxGroups];
};
// bytes of the K-split partial sums of a plan
inline size_t ad_m2l_partial_bytes(const AdM2LPlan &pl, int P) {
    return pl.nsplit > 1 ? sizeof(double) * (size_t)pl.nsplit * pl.units * 128 * P * P : 0;
}
// evaluation (FP64, box-id-indexed coefficient rows of stride coef_stride(P))
// adj = 1 in the transposed chain: P2M as the transpose of L2P (times 2^l),
// P2L as that of M2P (times 2^l of the box), L2P and M2P as those of P2M
// and P2L with their position derivatives (outputs times 2^-l)
hipError_t ad_launch_p2m(int P, int64_t nleaf, const int *lbox, const uint32_t *lstart, const uint8_t *llev, int adj,
                         const double4 *rec, double *M, bool f32, hipStream_t st);
hipError_t ad_launch_m2m(int P, int64_t b0, int64_t nb, const uint8_t *leaf, const int *child, const double *tab,
                         double *M, hipStream_t st);
// mixed form: the per-level maxima of |M_c rho_inv[c]| over the boxes of
// levels >= 2 (lmax, kLevelSlots words, zeroed beforehand), then the scaled
// multipoles split into binary16 parts Bh [nbox + 1][S/8][hi8, lo8] (rows
// box2 .. nbox, the last all zero)
hipError_t ad_launch_pack_h(int P, int64_t box2, int64_t nbox, const int *lev, const double *M,
                            const float *rho_inv, uint32_t *lmax, void *Bh, hipStream_t st);
// M2L over the V slots in the binary16 encoding (3 products on the 16-bit
// matrix cores, FP32 accumulation merged into FP64), added into Lc
hipError_t ad_launch_m2l_h(int P, const AdM2LPlan &pl, const uint16_t *Ah, size_t astride, const int2 *cls,
                           const void *Bh, const int *vidx, int64_t box2, const int *tgt, int64_t zero_row,
                           const uint32_t *lmax, const float *oscale, double *Lc, double *partial, hipStream_t st);
// adds M2L over the V slots into Lc; with pl.nsplit > 1 through `partial`
// (ad_m2l_partial_bytes) and a summing kernel, in a fixed order
hipError_t ad_launch_m2l(int P, const AdM2LPlan &pl, const double *A, const int2 *cls, const double *M,
                         const int *vidx, int64_t box2, const int *tgt, int64_t zero_row, double *Lc, double *partial,
                         hipStream_t st);
hipError_t ad_launch_p2l(int P, int64_t nbox, const uint32_t *ox, const int *ix, const int *lev,
                         const uint32_t *code, const uint32_t *ps, const uint32_t *pe, int adj, const double4 *rec,
                         double *Lc, bool f32, hipStream_t st);
hipError_t ad_launch_l2l(int P, int64_t b0, int64_t nb, const uint32_t *code, const int *parent, const double *tab,
                         double *Lc, hipStream_t st);
hipError_t ad_launch_l2p(int P, int64_t nleaf, const int *lbox, const uint32_t *lstart, const uint8_t *llev,
                         int adj, const double4 *rec, const double *Lc, double4 *out, bool f32, hipStream_t st);
// one wave per P2P work unit (see ad_launch_units)
hipError_t ad_launch_m2p(int P, int64_t max_units, const uint32_t *nunits, const int2 *units, int adj,
                         const int *lbox, const uint32_t *lstart, const uint32_t *ow, const int *iw, const int *lev,
                         const uint32_t *code, const double4 *rec, const double *M, double4 *out, bool f32,
                         hipStream_t st);
// Work units of up to 64 targets, in two orders (units for P2P over U, with
// ou the U offsets; units_m for M2P over W, with ow the W offsets): pass 0
// counts per leaf into cnt (2 kAdUnitClasses nleaf words: per order, one
// run of leaves per class of unit weight, heaviest first), pass 1 fills both
// copies (leaf, first target) from uoff, the scan of those counts (the
// number of units at uoff[kAdUnitClasses nleaf]), reading each leaf's
// classes back from cnt
constexpr int kAdUnitClasses = 8;
hipError_t ad_launch_units(int64_t nleaf, int pass, const uint32_t *lstart, const int *lbox, const uint32_t *ou,
                           const uint32_t *ow, const int *iu, const uint32_t *ps, const uint32_t *pe, uint32_t *cnt,
                           const uint32_t *uoff, int2 *units, int2 *units_m, hipStream_t st);
// one wave per unit; max_units bounds *nunits (the grid's size)
// with fuse non-NULL the kernel ends with the combine (no near partials);
// f32: the pair arithmetic in FP32 (the mixed form)
hipError_t ad_launch_p2p(int64_t max_units, const uint32_t *nunits, const int2 *units, const int *lbox,
                         const uint32_t *lstart, const uint32_t *ou, const int *iu, const int *lev, const uint32_t *code,
                         const uint32_t *ps, const uint32_t *pe, const double4 *rec, double4 *out, const Combine *fuse,
                         bool f32, hipStream_t st);

// scratch.hip: device address of the current device's static scratch array
// (FMM_NOALLOC_SCRATCH_BYTES), looked up on the first call per device
hipError_t noalloc_scratch(void **ptr);

// m2l.hip: every level 2..L in one launch; B[l], Lc[l] indexed by level.
// Mixed form: A = bf16 operator parts spaced astride elements apart (layout
// [part][317][R/16][S/8][16][8]), B[l] = FP32 padded multipole grid.  Both
// forms cut the small levels into K parts: `partial` >= m2l_partial_bytes()
// of FP64 scratch.
size_t m2l_partial_bytes(int P, int L, bool f64, int ncu);
constexpr int kMixedSplit3PMax = 13;  // LDS holds the 3-part operator ring up to p = 13
// The 2-part bf16 split (about 16 bits per operand) keeps the mixed force
// within 1e-6 of the FP64 form up to p = 10 only (measured 1.2e-6 at
// p = 11 and 16).
constexpr int kMixedSplit2PMax = 10;
// Binary16 encoding of the mixed form (half != NULL): A = the two binary16
// parts of a_r T rho_c (same layout as the bf16 parts), B[l] = the pack
// kernel's binary16 parts of the multipoles times 1/rho_c and the level
// scale 2^e_l; row r of the result is multiplied by oscale[r] 2^-e_l, with
// oscale[r] = 1/a_r.
struct M2LHalf {
    const uint32_t *lmax;   // per-level maxima (by level) of the scaled multipoles
    const float *oscale;    // [S]
};
hipError_t launch_m2l(int P, int L, bool f64, int nsplit, void *const *B, void *const *Lc,
                      const int *out_f64, const void *A, size_t astride, const int2 *cls,
                      double *partial, size_t partial_bytes, int ncu, const M2LHalf *half,
                      hipStream_t st);

}  // namespace fmm

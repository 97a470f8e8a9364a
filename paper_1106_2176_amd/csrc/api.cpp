// api.cpp -- the C ABI (include/fmm.h): validation, memory, level selection,
// operator tables and the order of kernel launches.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "opgen.hpp"

using namespace fmm;

namespace {

thread_local std::string g_err;

fmm_status fail(fmm_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(FMM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));       \
    } while (0)

// ------------------------------------------------------------- allocation
struct Alloc {
    fmm_alloc_fn fa = nullptr;
    fmm_free_fn ff = nullptr;
    void *ctx = nullptr;
};

void ensure_pool(int dev) {
    static std::mutex mu;
    static std::vector<int> done;
    std::lock_guard<std::mutex> g(mu);
    for (int d : done)
        if (d == dev) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    done.push_back(dev);
}

struct Buf {
    void *p = nullptr;
    size_t cap = 0;
};

// ------------------------------------------------------------ operators
struct Ops {
    int p = 0;
    // [8][P2][P2] input-major transfer tables
    double *up64 = nullptr, *down64 = nullptr, *aup64 = nullptr, *adown64 = nullptr;
    float *up32 = nullptr, *down32 = nullptr, *aup32 = nullptr, *adown32 = nullptr;
    // M2L tables (316 operators + a zero one): FP64 [317][R][S], and three
    // bf16 parts [3][317][R/16][S/8][16][8] for the mixed form (a 16-row tile
    // stored piece by piece, so that the mixed kernel's copy of four pieces
    // of a row tile reads one contiguous kilobyte); forward and adjoint
    double *m2l64 = nullptr, *am2l64 = nullptr;
    uint16_t *m2lbf = nullptr, *am2lbf = nullptr;
    size_t bf_part = 0;  // elements per bf16 (and binary16) part
    // binary16 encoding: a_r T rho_c in two binary16 parts, same layout as
    // the bf16 parts, with rho_c the harmonic size of coefficient c's degree
    // and a_r a power of two per row and table; rho_inv[c] = 1 / rho_c (the
    // pack's scale), oscale / aoscale[r] = 1 / a_r of the forward / adjoint
    // table (the M2L output's)
    uint16_t *m2lh = nullptr, *am2lh = nullptr;
    float *rho_inv = nullptr, *oscale = nullptr, *aoscale = nullptr;
    // rotation-based M2L (FP64 form), compact per offset id (made on first
    // use): forward D of offset -d and Tz, adjoint D of offset d and Tz^T
    double *rot64 = nullptr, *tz64 = nullptr, *arot64 = nullptr, *atz64 = nullptr;
    int2 *cls = nullptr; // [8][189] (packed source offset, table id)
};

std::mutex g_ops_mu;
std::map<std::pair<int, int>, Ops *> g_ops;

int id316_of(int dx, int dy, int dz) {
    static int tab[343];
    static bool init = false;
    if (!init) {
        int c = 0;
        for (int i = 0; i < 343; ++i) {
            const int ox = i % 7 - 3, oy = (i / 7) % 7 - 3, oz = i / 49 - 3;
            const int m = std::max(std::abs(ox), std::max(std::abs(oy), std::abs(oz)));
            tab[i] = m >= 2 ? c++ : -1;
        }
        init = true;
    }
    return tab[offset_id343(dx, dy, dz)];
}

fmm_status build_ops(int p, Ops **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_ops_mu);
    auto it = g_ops.find({dev, p});
    if (it != g_ops.end()) {
        *out = it->second;
        return FMM_OK;
    }
    const int P2 = p * p, R = m2l_rows(p), S = coef_stride(p);
    Ops *o = new Ops();
    o->p = p;
    std::vector<double> mat((size_t)P2 * P2);
    std::vector<double> up((size_t)8 * P2 * P2), down(up.size()), aup(up.size()), adown(up.size());
    for (int c = 0; c < 8; ++c) {
        op_m2m(p, c, mat.data());  // A_c [out][in]
        for (int i = 0; i < P2; ++i)
            for (int j = 0; j < P2; ++j) {
                up[((size_t)c * P2 + j) * P2 + i] = mat[(size_t)i * P2 + j];     // [c][in][out]
                adown[((size_t)c * P2 + i) * P2 + j] = mat[(size_t)i * P2 + j];  // A_c^T
            }
        op_l2l(p, c, mat.data());  // B_c [out][in]
        for (int i = 0; i < P2; ++i)
            for (int j = 0; j < P2; ++j) {
                down[((size_t)c * P2 + j) * P2 + i] = mat[(size_t)i * P2 + j];
                aup[((size_t)c * P2 + i) * P2 + j] = mat[(size_t)i * P2 + j];  // B_c^T
            }
    }
    // 316 operators plus one all-zero operator (id 316) that kernels read
    // for K pieces past the end of a class's list
    const size_t nT = (size_t)(kNumOffsets + 1) * R * S;
    std::vector<double> f64(nT, 0.0), af64(nT, 0.0);
    for (int i = 0; i < 343; ++i) {
        const int dx = i % 7 - 3, dy = (i / 7) % 7 - 3, dz = i / 49 - 3;
        const int id = id316_of(dx, dy, dz);
        if (id < 0) continue;
        // forward: source at t + d, operator for offset (target - source) = -d
        op_m2l(p, -dx, -dy, -dz, mat.data());
        for (int r = 0; r < P2; ++r)
            for (int c = 0; c < P2; ++c) f64[((size_t)id * R + r) * S + c] = mat[(size_t)r * P2 + c];
        // adjoint: transpose of the operator for offset d
        op_m2l(p, dx, dy, dz, mat.data());
        for (int r = 0; r < P2; ++r)
            for (int c = 0; c < P2; ++c) af64[((size_t)id * R + r) * S + c] = mat[(size_t)c * P2 + r];
    }
    std::vector<int2> cls((size_t)8 * kOffsetsPerClass);
    for (int k = 0; k < 8; ++k) {
        const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
        int s = 0;
        for (int dz = -2 - kz; dz <= 3 - kz; ++dz)
            for (int dy = -2 - ky; dy <= 3 - ky; ++dy)
                for (int dx = -2 - kx; dx <= 3 - kx; ++dx) {
                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                    int2 e;
                    e.x = (dx + 4) | ((dy + 4) << 4) | ((dz + 4) << 8);
                    e.y = id316_of(dx, dy, dz);
                    cls[(size_t)k * kOffsetsPerClass + s++] = e;
                }
    }
    auto up32f = [](const std::vector<double> &v) {
        std::vector<float> f(v.size());
        for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
        return f;
    };
    auto upload = [](void **dst, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return e;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    const size_t tb = up.size();
    hipError_t e = hipSuccess;
    std::vector<float> t32;
#define UP64(field, vec) \
    if (e == hipSuccess) e = upload((void **)&o->field, vec.data(), vec.size() * sizeof(vec[0]));
    // the transfer kernels read up to 4 p^2 + 16 entries past a table's end:
    // rows of the last row tile past p^2 (whose results are discarded) and K
    // steps past p^2 (multiplied by zero)
    for (auto *v : {&up, &down, &aup, &adown}) v->resize(v->size() + 4 * (size_t)P2 + 16, 0.0);
    UP64(up64, up) UP64(down64, down) UP64(aup64, aup) UP64(adown64, adown)
    t32 = up32f(up); UP64(up32, t32)
    t32 = up32f(down); UP64(down32, t32)
    t32 = up32f(aup); UP64(aup32, t32)
    t32 = up32f(adown); UP64(adown32, t32)
    std::vector<uint16_t> fbf(3 * nT), afbf(3 * nT);
    const int PPO = S / 8;
    for (size_t i = 0; i < nT; ++i) {
        const size_t id = i / ((size_t)R * S), rem = i % ((size_t)R * S);
        const int row = (int)(rem / S), col = (int)(rem % S);
        const size_t j = id * R * S + (((size_t)(row / 16) * PPO + col / 8) * 16 + row % 16) * 8 + col % 8;
        uint16_t pt[3];
        split_bf16(f64[i], 3, pt);
        for (int k = 0; k < 3; ++k) fbf[k * nT + j] = pt[k];
        split_bf16(af64[i], 3, pt);
        for (int k = 0; k < 3; ++k) afbf[k * nT + j] = pt[k];
    }
    UP64(m2l64, f64) UP64(am2l64, af64) UP64(m2lbf, fbf) UP64(am2lbf, afbf)
    UP64(cls, cls)
    {
        // binary16 tables: columns scaled by the harmonic size rho_c of their
        // degree (the multipoles are divided by it), each row by the power of
        // two a_r that puts the row's largest entry just below 2^14, so that
        // the low part of every entry that matters stays a normal binary16
        // number and no entry overflows (binary16 ends at 65520)
        double rho[FMM_P_MAX];
        harmonic_scale(p, rho);
        std::vector<double> rc(S, 0.0);
        std::vector<float> rinv(S, 0.0f), osc(S, 0.0f), aosc(S, 0.0f);
        for (int c = 0; c < P2; ++c) {
            int n = 0;
            while ((n + 1) * (n + 1) <= c) ++n;
            rc[c] = rho[n];
            rinv[c] = (float)(1.0 / rho[n]);
        }
        auto encode = [&](const std::vector<double> &tab, std::vector<uint16_t> &out,
                          std::vector<float> &oscale) {
            std::vector<double> a(R, 0.0);
            for (int r = 0; r < P2; ++r) {
                double mx = 0.0;
                for (size_t id = 0; id < (size_t)kNumOffsets; ++id)
                    for (int c = 0; c < P2; ++c)
                        mx = std::max(mx, std::fabs(tab[(id * R + r) * S + c]) * rc[c]);
                int ex = 0;
                (void)std::frexp(mx, &ex);  // mx < 2^ex
                a[r] = mx > 0.0 ? std::ldexp(1.0, 14 - ex) : 1.0;
                oscale[r] = (float)(1.0 / a[r]);
            }
            out.assign(2 * nT, 0);
            for (size_t i = 0; i < nT; ++i) {
                const size_t id = i / ((size_t)R * S), rem = i % ((size_t)R * S);
                const int row = (int)(rem / S), col = (int)(rem % S);
                const size_t j = id * R * S + (((size_t)(row / 16) * PPO + col / 8) * 16 + row % 16) * 8 + col % 8;
                uint16_t pt[2];
                split_f16(tab[i] * a[row] * rc[col], pt);
                out[j] = pt[0];
                out[nT + j] = pt[1];
            }
        };
        std::vector<uint16_t> fh, afh;
        encode(f64, fh, osc);
        encode(af64, afh, aosc);
        UP64(m2lh, fh) UP64(am2lh, afh) UP64(rho_inv, rinv) UP64(oscale, osc) UP64(aoscale, aosc)
    }
#undef UP64
    (void)tb;
    if (e != hipSuccess) return fail(FMM_EDEVICE, std::string("operator upload: ") + hipGetErrorString(e));
    o->bf_part = nT;
    g_ops[{dev, p}] = o;
    *out = o;
    return FMM_OK;
}

// Tables of the rotation-based M2L for p (FP64 form): for every M2L offset
// id, D and Tz of op_m2l_rotated in the compact layouts of rot_deg_off and
// tz_off.  The forward pair (target t, source t + d) takes the operator of
// offset -d; the adjoint takes the transpose of the operator of offset d,
// D_d^T Tz^T D_d.  Each rotation needs a quadrature over the sphere, so the
// offsets are spread over host threads.
fmm_status build_rot_ops(int p, Ops *o) {
    std::lock_guard<std::mutex> g(g_ops_mu);
    if (o->rot64) return FMM_OK;
    const int P2 = p * p, ND = rot_size(p), NZ = tz_size(p);
    const size_t nid = (size_t)kNumOffsets;
    std::vector<double> fr(nid * ND), ft(nid * NZ), ar(nid * ND), at(nid * NZ);
    std::vector<int> todo;
    for (int i = 0; i < 343; ++i)
        if (id316_of(i % 7 - 3, (i / 7) % 7 - 3, i / 49 - 3) >= 0) todo.push_back(i);
    auto compact = [&](const double *D, const double *Tz, bool transpose_tz, double *dr, double *dt) {
        for (int n = 0; n < p; ++n) {
            const int w = 2 * n + 1, b = n * n;
            for (int r = 0; r < w; ++r)
                for (int c = 0; c < w; ++c) dr[rot_deg_off(n) + r * w + c] = D[(size_t)(b + r) * P2 + b + c];
        }
        for (int m = 0; m < p; ++m)
            for (int kind = 0; kind < (m == 0 ? 1 : 2); ++kind) {
                const int w = p - m;
                for (int kk = m; kk < p; ++kk)
                    for (int nn = m; nn < p; ++nn) {
                        const int ro = kk * kk + (m == 0 ? 0 : 2 * m - 1 + kind);
                        const int ci = nn * nn + (m == 0 ? 0 : 2 * m - 1 + kind);
                        const double v = transpose_tz ? Tz[(size_t)ci * P2 + ro] : Tz[(size_t)ro * P2 + ci];
                        dt[tz_off(p, m, kind) + (kk - m) * w + (nn - m)] = v;
                    }
            }
    };
    auto work = [&](size_t first, size_t step) {
        std::vector<double> D((size_t)P2 * P2), Tz((size_t)P2 * P2);
        for (size_t j = first; j < todo.size(); j += step) {
            const int i = todo[j];
            const int dx = i % 7 - 3, dy = (i / 7) % 7 - 3, dz = i / 49 - 3;
            const size_t id = (size_t)id316_of(dx, dy, dz);
            op_m2l_rotated(p, -dx, -dy, -dz, D.data(), Tz.data());
            compact(D.data(), Tz.data(), false, &fr[id * ND], &ft[id * NZ]);
            op_m2l_rotated(p, dx, dy, dz, D.data(), Tz.data());
            compact(D.data(), Tz.data(), true, &ar[id * ND], &at[id * NZ]);
        }
    };
    const size_t nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (size_t t = 1; t < nth; ++t) th.emplace_back(work, t, nth);
    work(0, nth);
    for (auto &x : th) x.join();
    auto upload = [](double **dst, const std::vector<double> &v) -> hipError_t {
        hipError_t e = hipMalloc((void **)dst, v.size() * sizeof(double));
        if (e != hipSuccess) return e;
        return hipMemcpy(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice);
    };
    double *d1 = nullptr, *d2 = nullptr, *d3 = nullptr, *d4 = nullptr;
    hipError_t e = upload(&d1, fr);
    if (e == hipSuccess) e = upload(&d2, ft);
    if (e == hipSuccess) e = upload(&d3, ar);
    if (e == hipSuccess) e = upload(&d4, at);
    if (e != hipSuccess) return fail(FMM_EDEVICE, std::string("rotation table upload: ") + hipGetErrorString(e));
    o->tz64 = d2;
    o->arot64 = d3;
    o->atz64 = d4;
    o->rot64 = d1;
    return FMM_OK;
}

constexpr int kStages = 9;
constexpr int kTimeRing = 32;  // event sets: stage times of the last 32 profiled calls
constexpr int kEvents = kStages + 3;  // stage boundaries + start/end of a concurrent P2P

// An instantiated graph of one evaluate or backward chain and the arguments
// it was captured with (graph mode).
struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;  // stream of its latest launch
    uint64_t gen = 0;            // tree memory generation at capture
    int L = -1;
    int64_t n = 0;
    fmm_config cfg{};
    const void *arg[5] = {};
    int32_t flags = 0;
};

// Adaptive tree (cfg.adaptive): box arrays indexed by global box id (levels
// concatenated breadth first), the U/W/X lists in CSR form, the V lists as
// 189 slots per box of level >= 2, the leaves in particle order, and host
// copies of the level offsets and of the M2L target groups.
constexpr int kAdHostWords = 128;  // 4 totals + 8 groups per level 2..10
struct AdTree {
    int depth = 0;
    int64_t nbox = 0, nleaf = 0, nvbox = 0;  // nvbox: boxes of levels >= 2
    int64_t off[FMM_MAX_LEVEL + 2] = {};      // first box of each level, off[depth + 1] = nbox
    int64_t nlist[3] = {};                    // items of U, W, X
    int64_t goff[8 * FMM_MAX_LEVEL + 1] = {}; // first target of each (level, class) group
    AdM2LPlan plan{};
    uint32_t *hbuf = nullptr;                 // pinned host words for the build's counts
    Buf code, ps, pe, parent, child, leaf, cmask, nchild, coff, lev, col, vidx, cnts, offs, iu, iw, ix,
        is_head, head, hoff, lbox, lstart, llev, tgt, ccnt, goffd, offd, ucnt, uoff, units, s27, units_m;
    Buf skey, cstart, ks_a, ks_b, ks_v, ks_h;  // the key sort: sorted keys, coarse starts, scratch
    int64_t max_units = 0;  // bound of the P2P work units (their count stays on the device)
    std::vector<Buf *> bufs() {
        return {&code, &ps, &pe, &parent, &child, &leaf, &cmask, &nchild, &coff, &lev, &col, &vidx, &cnts,
                &offs, &iu, &iw, &ix, &is_head, &head, &hoff, &lbox, &lstart, &llev, &tgt, &ccnt, &goffd,
                &offd, &ucnt, &uoff, &units, &s27, &skey, &cstart, &ks_a, &ks_b, &ks_v, &ks_h, &units_m};
    }
};

}  // namespace

struct fmm_tree {
    fmm_config cfg;
    int dtype = FMM_F64;
    int64_t n = 0;
    int L = 0;
    int64_t nleaf = 1;
    int64_t max_count = 0;
    int dev = 0;
    int ncu = 0;  // compute units of the device
    hipStream_t stream = nullptr;
    Alloc al;
    Buf key10, rank, cnt, start, tmp, perm, scan, counters, xyz32, xyz64, nearf, farf, pairs, m2lpart,
        lmax;
    hipEvent_t ev_counters = nullptr;  // after the copy of the build counters
    Buf M[FMM_MAX_LEVEL + 1], Lc[FMM_MAX_LEVEL + 1], pack[FMM_MAX_LEVEL + 1];
    unsigned int *host_counters = nullptr;  // pinned [4]
    unsigned int *host_counters_dev = nullptr;  // their address for kernels
    Ops *ops = nullptr;
    hipEvent_t ev[kTimeRing][kEvents] = {};
    bool p2p_side[kTimeRing] = {};  // the call's P2P ran on the side stream
    bool ev_ready = false;
    hipStream_t side = nullptr;         // stream of the concurrent near field
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int64_t ncalls = 0;  // profiled calls since the last reset
    int cur = 0;         // event set of the call in progress
    uint64_t gen = 0;    // bumped whenever a buffer is allocated or released
    hipStream_t cap = nullptr;  // capture stream of graph mode
    bool capturing = false;
    GraphSlot gfwd, gbwd;       // graphs of fmm_evaluate and fmm_backward
    bool quiet = false;         // a call that records no profiling events
    AdTree *ad = nullptr;       // the adaptive tree (cfg.adaptive), else NULL
};

namespace {

// Device buffers of one evaluate or backward call: taken from the tree's
// workspace (fmm_evaluate, fmm_backward) or carved from the library's static
// scratch array (fmm_evaluate_noalloc).
struct Work {
    double4 *nearf = nullptr, *farf = nullptr;  // near / far partial results, sorted order
    void *M[FMM_MAX_LEVEL + 1] = {}, *Lc[FMM_MAX_LEVEL + 1] = {};  // coefficient grids
    void *pack[FMM_MAX_LEVEL + 1] = {};                            // M2L operand grids
    double *m2lpart = nullptr;                                     // M2L K-split partial sums
    size_t m2lpart_bytes = 0;
    uint32_t *lmax = nullptr;  // per-level maxima of the binary16 M2L encoding
};

bool is_f64_form(const fmm_tree *t) { return t->cfg.precision == FMM_PREC_FP64; }

// the mixed form's M2L in the binary16 encoding
bool m2l_half(const fmm_config &c) { return c.precision == FMM_PREC_MIXED && c.m2l_fp16 != 0; }

// bf16 parts of the mixed M2L (0 selects the default, 3)
int split_parts(const fmm_config &c) { return c.bf16_splits == 2 ? 2 : 3; }

// Storage precision of the coefficients of level l: FP64 in the plain form;
// in the mixed form FP64 for coarse levels (<= 4096 boxes) except the leaf
// level, whose multipoles and locals are produced and consumed by the FP32
// P2M and L2P kernels together with the FP32 particle layout.
int level_f64(const fmm_tree *t, int l) {
    if (is_f64_form(t)) return 1;
    return (l <= 4 && l != t->L) ? 1 : 0;
}

// Byte sizes of the per-call buffers (the far-field ones are zero without a
// far field, L < 2).
struct WorkSizes {
    size_t nearf = 0, farf = 0, m2lpart = 0, lmax = 0;
    size_t M[FMM_MAX_LEVEL + 1] = {}, Lc[FMM_MAX_LEVEL + 1] = {}, pack[FMM_MAX_LEVEL + 1] = {};
};

WorkSizes work_sizes(const fmm_tree *t, bool far) {
    WorkSizes z;
    const int P = t->cfg.p, S = coef_stride(P), L = t->L;
    const bool f64 = is_f64_form(t);
    z.nearf = sizeof(double4) * (size_t)t->n;
    if (!far || L < 2) return z;
    if (t->ad) {  // FP64 coefficients by box id, plus the zero row
        z.farf = sizeof(double4) * (size_t)t->n;
        z.M[0] = z.Lc[0] = sizeof(double) * (size_t)(t->ad->nbox + 1) * S;
        z.m2lpart = ad_m2l_partial_bytes(t->ad->plan, P);
        if (m2l_half(t->cfg)) {  // the binary16 parts of the multipoles, and the level maxima
            z.pack[0] = sizeof(float) * (size_t)(t->ad->nbox + 1) * S;
            z.lmax = sizeof(uint32_t) * kLevelSlots;
        }
        return z;
    }
    z.farf = sizeof(double4) * (size_t)t->n;
    for (int l = 2; l <= L; ++l) {
        const size_t nb = (size_t)1 << (3 * l);
        const size_t es = level_f64(t, l) ? 8 : 4;
        z.M[l] = z.Lc[l] = nb * S * es;
        const size_t g = ((size_t)1 << l) + 6;
        z.pack[l] = g * g * g * S * (f64 ? 8 : 4);
    }
    z.m2lpart = m2l_partial_bytes(P, L, f64, t->ncu);
    if (m2l_half(t->cfg)) z.lmax = sizeof(uint32_t) * kLevelSlots;
    return z;
}

fmm_status ensure(fmm_tree *t, Buf &b, size_t bytes, hipStream_t st) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return FMM_OK;
    // a graph is captured right after an eager run of the same chain, which
    // allocated everything it needs
    if (t->capturing) return fail(FMM_EDEVICE, "internal: allocation during graph capture");
    ++t->gen;
    if (b.p) {
        if (t->al.fa)
            t->al.ff(b.p, st, t->al.ctx);
        else
            (void)hipFreeAsync(b.p, st);
        b.p = nullptr;
        b.cap = 0;
    }
    void *p = nullptr;
    if (t->al.fa) {
        p = t->al.fa(bytes, st, t->al.ctx);
        if (!p) return fail(FMM_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        hipError_t e = hipMallocAsync(&p, bytes, st);
        if (e != hipSuccess || !p)
            return fail(FMM_ENOMEM, "hipMallocAsync(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    b.p = p;
    b.cap = bytes;
    return FMM_OK;
}

void release(fmm_tree *t, Buf &b, hipStream_t st) {
    if (!b.p) return;
    ++t->gen;
    if (t->al.fa)
        t->al.ff(b.p, st, t->al.ctx);
    else
        (void)hipFreeAsync(b.p, st);
    b.p = nullptr;
    b.cap = 0;
}

fmm_status validate_cfg(const fmm_config *c) {
    if (!c) return fail(FMM_EINVAL, "config is NULL");
    if (c->abi_version != FMM_ABI_VERSION) return fail(FMM_EINVAL, "ABI version mismatch");
    if (c->p < 1 || c->p > FMM_P_MAX) return fail(FMM_EINVAL, "p must be in [1, 16]");
    if (c->leaf_max < 1) return fail(FMM_EINVAL, "leaf_max must be >= 1");
    if (c->max_level < 0 || c->max_level > FMM_MAX_LEVEL) return fail(FMM_EINVAL, "max_level must be in [0, 10]");
    if (c->precision != FMM_PREC_FP64 && c->precision != FMM_PREC_MIXED)
        return fail(FMM_EINVAL, "unknown precision");
    if (c->bf16_splits != 0 && c->bf16_splits != 2 && c->bf16_splits != 3)
        return fail(FMM_EINVAL, "bf16_splits must be 0, 2 or 3");
    const bool bf16 = c->precision == FMM_PREC_MIXED && !c->m2l_fp16;
    if (bf16 && c->bf16_splits != 2 && c->p > kMixedSplit3PMax)
        return fail(FMM_EUNSUPPORTED, "the mixed form with a 3-part split supports p <= 13");
    if (bf16 && c->bf16_splits == 2 && c->p > kMixedSplit2PMax)
        return fail(FMM_EUNSUPPORTED, "the mixed form with a 2-part bf16 split supports p <= 10 "
                                      "(above it the force misses the 1e-6 budget)");
    if (!(c->box_size > 0.0) || !std::isfinite(c->box_size)) return fail(FMM_EINVAL, "box_size must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c->box_lo[a])) return fail(FMM_EINVAL, "box_lo must be finite");
    if (c->graph && c->profile) return fail(FMM_EINVAL, "graph and profile are exclusive");
    if (c->m2l_rotation && c->precision != FMM_PREC_FP64)
        return fail(FMM_EINVAL, "the rotation-based M2L is an option of the FP64 form");
    if (c->m2l_rotation && c->p < 2) return fail(FMM_EINVAL, "the rotation-based M2L needs p >= 2");
    if (c->adaptive && c->precision == FMM_PREC_MIXED && !c->m2l_fp16)
        return fail(FMM_EUNSUPPORTED, "the adaptive tree's mixed form uses the binary16 M2L (m2l_fp16 = 1)");
    if (c->adaptive && c->m2l_rotation)
        return fail(FMM_EUNSUPPORTED, "the adaptive tree uses the dense M2L only");
    if (c->profile_stages >> kStages) return fail(FMM_EINVAL, "profile_stages has bits past stage 8");
    if ((c->alloc == nullptr) != (c->free == nullptr))
        return fail(FMM_EINVAL, "alloc and free callbacks must be given together");
    return FMM_OK;
}

bool stage_on(const fmm_tree *t, int i) {
    return t->cfg.profile_stages == 0 || ((t->cfg.profile_stages >> i) & 1u);
}

// Event at stage boundary b (start of stage b, end of stage b - 1), or at the
// start / end (kStages + 1 / + 2) of a P2P on the side stream; only where a
// selected stage begins or ends.
fmm_status rec(fmm_tree *t, int stage, hipStream_t st) {
    if (!t->cfg.profile || t->capturing || t->quiet) return FMM_OK;
    const bool want = stage > kStages ? stage_on(t, 7)
                                      : (stage < kStages && stage_on(t, stage)) ||
                                            (stage > 0 && stage_on(t, stage - 1));
    if (!want) return FMM_OK;
    if (!t->ev_ready) {
        for (int j = 0; j < kTimeRing; ++j)
            for (int i = 0; i < kEvents; ++i) HIPCHK(hipEventCreate(&t->ev[j][i]));
        t->ev_ready = true;
    }
    HIPCHK(hipEventRecord(t->ev[t->cur][stage], st));
    return FMM_OK;
}

#define CHK(x)                           \
    do {                                 \
        fmm_status s_ = (x);             \
        if (s_ != FMM_OK) return s_;     \
    } while (0)

// Per-call buffers from the tree's workspace, grown through its allocator.
fmm_status work_from_tree(fmm_tree *t, bool far, hipStream_t st, Work &w) {
    const WorkSizes z = work_sizes(t, far);
    CHK(ensure(t, t->nearf, z.nearf, st));
    w.nearf = (double4 *)t->nearf.p;
    if (!z.farf) return FMM_OK;
    CHK(ensure(t, t->farf, z.farf, st));
    w.farf = (double4 *)t->farf.p;
    for (int l = 0; l <= FMM_MAX_LEVEL; ++l) {
        if (z.M[l]) {
            CHK(ensure(t, t->M[l], z.M[l], st));
            CHK(ensure(t, t->Lc[l], z.Lc[l], st));
            w.M[l] = t->M[l].p;
            w.Lc[l] = t->Lc[l].p;
        }
        if (z.pack[l]) {
            CHK(ensure(t, t->pack[l], z.pack[l], st));
            w.pack[l] = t->pack[l].p;
        }
    }
    if (z.m2lpart) {
        CHK(ensure(t, t->m2lpart, z.m2lpart, st));
        w.m2lpart = (double *)t->m2lpart.p;
        w.m2lpart_bytes = t->m2lpart.cap;
    }
    if (z.lmax) {
        CHK(ensure(t, t->lmax, z.lmax, st));
        w.lmax = (uint32_t *)t->lmax.p;
    }
    return FMM_OK;
}

// Per-call buffers carved, 256-byte aligned, from the static scratch array
// of the current device (FMM_NOALLOC_SCRATCH_BYTES).  Nothing in them needs
// clearing: every kernel writes each element before any kernel reads it.
fmm_status work_from_scratch(fmm_tree *t, bool far, Work &w) {
    const WorkSizes z = work_sizes(t, far);
    size_t off = 0;
    auto take = [&](size_t bytes) -> size_t {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_near = take(z.nearf), o_far = take(z.farf), o_part = take(z.m2lpart),
                 o_lmax = take(z.lmax);
    size_t oM[FMM_MAX_LEVEL + 1] = {}, oL[FMM_MAX_LEVEL + 1] = {}, oP[FMM_MAX_LEVEL + 1] = {};
    for (int l = 0; l <= FMM_MAX_LEVEL && z.farf; ++l) {
        if (z.M[l]) {
            oM[l] = take(z.M[l]);
            oL[l] = take(z.Lc[l]);
        }
        if (z.pack[l]) oP[l] = take(z.pack[l]);
    }
    if (off > (size_t)FMM_NOALLOC_SCRATCH_BYTES)
        return fail(FMM_EINVAL, "this tree's evaluation needs " + std::to_string(off) +
                                    " bytes of scratch, more than FMM_NOALLOC_SCRATCH_BYTES (" +
                                    std::to_string((size_t)FMM_NOALLOC_SCRATCH_BYTES) + ")");
    unsigned char *base = nullptr;
    HIPCHK(noalloc_scratch((void **)&base));
    w.nearf = (double4 *)(base + o_near);
    if (!z.farf) return FMM_OK;
    w.farf = (double4 *)(base + o_far);
    if (z.m2lpart) {
        w.m2lpart = (double *)(base + o_part);
        w.m2lpart_bytes = z.m2lpart;
    }
    if (z.lmax) w.lmax = (uint32_t *)(base + o_lmax);
    for (int l = 0; l <= FMM_MAX_LEVEL; ++l) {
        if (z.M[l]) {
            w.M[l] = base + oM[l];
            w.Lc[l] = base + oL[l];
        }
        if (z.pack[l]) w.pack[l] = base + oP[l];
    }
    return FMM_OK;
}

// The far + near chain shared by the forward evaluation and the adjoint.
// fuse: the combine of a forward evaluation, taken over by the last kernel
// (*fused is then set): P2P when it runs on the call's stream after the far
// field; L2P, after the join, when the near field runs on the side stream
// (forked beside M2L, it ends before the far field does)
fmm_status run_chain(fmm_tree *t, const Work &w, const void *charges, bool adjoint, bool do_far,
                     bool do_near, hipStream_t st, const Combine *fuse = nullptr, bool *fused = nullptr) {
    const int P = t->cfg.p, L = t->L;
    const bool f64 = is_f64_form(t);
    void *src = f64 ? t->xyz64.p : t->xyz32.p;
    const uint32_t *start = (const uint32_t *)t->start.p;
    const int nsplit = split_parts(t->cfg);
    t->cur = (int)(t->ncalls % kTimeRing);

    // guards: every buffer a kernel will touch holds what that kernel assumes
    const size_t src_bytes = (f64 ? sizeof(double4) : sizeof(int4)) * (size_t)t->n;
    if ((f64 ? t->xyz64.cap : t->xyz32.cap) < src_bytes || !src)
        return fail(FMM_EDEVICE, "internal: particle buffer does not match the form");
    if (t->start.cap < sizeof(uint32_t) * (size_t)(t->nleaf + 1) || t->perm.cap < sizeof(uint32_t) * (size_t)t->n)
        return fail(FMM_EDEVICE, "internal: tree buffers too small");
    if (L >= 2 && level_f64(t, L) != (int)f64)
        return fail(FMM_EDEVICE, "internal: leaf-level precision differs from the particle precision");
    CHK(rec(t, 0, st));
    const bool side = do_near && do_far && L >= 2 && t->cfg.overlap_near && !t->quiet;
    // The charges go into the sorted records before anything reads them:
    // by P2M when it runs first (far field, P2P after it), else by a gather.
    const bool p2m_gathers = do_far && L >= 2 && !side;
    if (!p2m_gathers)
        HIPCHK(launch_gather_q(t->n, t->dtype, f64, (const uint32_t *)t->perm.p, charges, src, st));
    // Near field concurrently with the far field: P2P needs only the sorted
    // particles and writes its own buffer, so it is forked onto the library's
    // side stream and joined back before the combine.  The fork comes after
    // the pack, when the M2L kernel is next on the call's stream: its blocks
    // (two waves per SIMD) are placed with the P2P waves filling what they
    // leave, where P2P forked earlier would hold every slot of the chip.
    t->p2p_side[t->cur] = side;
    if (side && !t->side) {
        HIPCHK(hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&t->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&t->ev_join, hipEventDisableTiming));
    }
    auto fork_near = [&]() -> fmm_status {
        HIPCHK(hipEventRecord(t->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(t->side, t->ev_fork, 0));
        CHK(rec(t, kStages + 1, t->side));
        HIPCHK(launch_p2p(L, f64, src, start, w.nearf, nullptr, t->side));
        CHK(rec(t, kStages + 2, t->side));
        HIPCHK(hipEventRecord(t->ev_join, t->side));
        return FMM_OK;
    };
    if (L >= 2 && do_far) {
        if (!t->ops) return fail(FMM_EDEVICE, "internal: the tree has no translation tables");
        const Ops *o = t->ops;
        if (!w.farf) return fail(FMM_EDEVICE, "internal: no far-field buffers");
        CHK(rec(t, 1, st));
        // P2M at the leaves (for the adjoint: L2P^T, the same sum with w)
        HIPCHK(launch_p2m(P, L, f64, src, start, w.M[L], 1.0,
                          p2m_gathers ? (const uint32_t *)t->perm.p : nullptr, charges, t->dtype,
                          w.lmax, st));
        CHK(rec(t, 2, st));
        // upward sweep (adjoint: L2L^T)
        for (int l = L - 1; l >= 2; --l)
            HIPCHK(launch_transfer(true, P, l, level_f64(t, l + 1), level_f64(t, l), w.M[l + 1],
                                   w.M[l], adjoint ? o->aup32 : o->up32,
                                   adjoint ? o->aup64 : o->up64, st));
        CHK(rec(t, 3, st));
        {
            PackPlan pk{};
            pk.nlev = L - 1;
            pk.lmax = w.lmax;
            pk.rho_inv = o->rho_inv;
            for (int l = 2; l <= L; ++l) {
                const int i = l - 2;
                const int64_t g = ((int64_t)1 << l) + 6;
                pk.level[i] = l;
                pk.in_f64[i] = level_f64(t, l);
                pk.in[i] = w.M[l];
                pk.out[i] = w.pack[l];
                pk.row0[i + 1] = pk.row0[i] + g * g;
            }
            HIPCHK(launch_pack(P, f64, pk, st));
        }
        CHK(rec(t, 4, st));
        if (side) CHK(fork_near());
        // M2L at every level >= 2 in one launch (the levels are independent)
        {
            void *Bp[FMM_MAX_LEVEL + 1] = {}, *Lp[FMM_MAX_LEVEL + 1] = {};
            int of64[FMM_MAX_LEVEL + 1] = {};
            for (int l = 2; l <= L; ++l) {
                Bp[l] = w.pack[l];
                Lp[l] = w.Lc[l];
                of64[l] = level_f64(t, l);
            }
            const bool half = m2l_half(t->cfg);
            if (f64 && t->cfg.m2l_rotation) {  // rotate, translate along z, rotate back
                if (!o->rot64) return fail(FMM_EDEVICE, "internal: no rotation tables");
                HIPCHK(launch_m2l_rot(P, L, Bp, Lp, adjoint ? o->arot64 : o->rot64,
                                      adjoint ? o->atz64 : o->tz64, o->cls, st));
            } else {  // dense products grouped by offset on the matrix cores
                const void *A = f64    ? (const void *)(adjoint ? o->am2l64 : o->m2l64)
                                : half ? (const void *)(adjoint ? o->am2lh : o->m2lh)
                                       : (const void *)(adjoint ? o->am2lbf : o->m2lbf);
                const M2LHalf hv{w.lmax, adjoint ? o->aoscale : o->oscale};
                HIPCHK(launch_m2l(P, L, f64, nsplit, Bp, Lp, of64, A, o->bf_part, o->cls, w.m2lpart,
                                  w.m2lpart_bytes, t->ncu, half ? &hv : nullptr, st));
            }
        }
        CHK(rec(t, 5, st));
        // downward sweep (adjoint: M2M^T)
        for (int l = 2; l < L; ++l)
            HIPCHK(launch_transfer(false, P, l, level_f64(t, l), level_f64(t, l + 1), w.Lc[l],
                                   w.Lc[l + 1], adjoint ? o->adown32 : o->down32,
                                   adjoint ? o->adown64 : o->down64, st));
        CHK(rec(t, 6, st));
        // L2P (adjoint: P2M^T with its position derivative)
        // leaf-level coefficients share the particle precision (level_f64)
        if (side && fuse) {
            Combine cf = *fuse;
            cf.farf = w.nearf;  // far + near in one pass, after the join
            HIPCHK(hipStreamWaitEvent(st, t->ev_join, 0));
            HIPCHK(launch_l2p(P, L, f64, src, start, w.Lc[L], w.farf, &cf, st));
            if (fused) *fused = true;
        } else {
            HIPCHK(launch_l2p(P, L, f64, src, start, w.Lc[L], w.farf, nullptr, st));
        }
    } else {
        for (int s = 1; s <= 6; ++s) CHK(rec(t, s, st));
    }
    CHK(rec(t, 7, st));
    if (side) {
        HIPCHK(hipStreamWaitEvent(st, t->ev_join, 0));
    } else if (do_near) {
        HIPCHK(launch_p2p(L, f64, src, start, w.nearf, fuse, st));
        if (fused) *fused = fuse != nullptr;
    } else {
        HIPCHK(launch_zero((uint32_t *)w.nearf, 8 * t->n, st));
    }
    CHK(rec(t, 8, st));
    return FMM_OK;
}

// ------------------------------------------------------------ adaptive tree
template <typename T>
T *bp(const Buf &b) { return (T *)b.p; }

// Build of an adaptive tree: keys and the counting sort at the finest level
// Lf = max_level; the boxes level by level (a box over leaf_max below Lf is
// split, its non-empty children appended in Morton order; one host read of
// the child count per level); then the levels, colleagues and V slots, the
// U/W/X counts and the leaf heads, one host read of their totals and of the
// M2L group sizes, and the lists, the leaf list, the leaf-relative records
// and the grouped M2L targets.
fmm_status build_adaptive(fmm_tree *t, int64_t n, int32_t dtype, const void *pos, hipStream_t st) {
    const fmm_config &c = t->cfg;
    const int Lf = c.max_level;
    if (!t->ad && !(t->ad = new (std::nothrow) AdTree())) return fail(FMM_ENOMEM, "host allocation failed");
    AdTree *a = t->ad;
    if (!a->hbuf) HIPCHK(hipHostMalloc((void **)&a->hbuf, kAdHostWords * sizeof(uint32_t)));
    // the finest keys are sorted themselves (no bin per key of level Lf, so
    // that the cost does not grow with 8^Lf); box ranges come from the
    // sorted keys through the first position of each key of level cl, the
    // first level with about as many keys as particles (at most 7)
    int cl = 0;
    while (cl < std::min(Lf, 7) && ((int64_t)1 << (3 * cl)) < n) ++cl;
    const int64_t nc = (int64_t)1 << (3 * cl), hw = key_sort_hist_words(n);
    // the boxes of a level l >= 1 are non-empty children of split boxes of
    // level l - 1, which are disjoint and hold more than leaf_max each
    int64_t bound = 0;
    for (int l = 0; l <= Lf; ++l) {
        int64_t b = std::min<int64_t>((int64_t)1 << (3 * l), n);
        if (l > 0) b = std::min<int64_t>(b, 8 * (n / ((int64_t)c.leaf_max + 1)));
        bound += b;
    }
    const size_t u4 = sizeof(uint32_t);
    CHK(ensure(t, t->key10, u4 * n, st));
    CHK(ensure(t, t->counters, 4 * u4, st));
    CHK(ensure(t, t->perm, u4 * n, st));
    CHK(ensure(t, t->xyz64, sizeof(double4) * n, st));
    CHK(ensure(t, t->scan, u4 * scan_scratch_words(bound + 1), st));
    CHK(ensure(t, a->skey, u4 * n, st));
    CHK(ensure(t, a->cstart, u4 * (nc + 1), st));
    CHK(ensure(t, a->ks_a, u4 * n, st));
    CHK(ensure(t, a->ks_b, u4 * n, st));
    CHK(ensure(t, a->ks_v, u4 * n, st));
    CHK(ensure(t, a->ks_h, u4 * (2 * hw + 1 + scan_scratch_words(hw)), st));
    CHK(ensure(t, a->code, u4 * bound, st));
    CHK(ensure(t, a->ps, u4 * bound, st));
    CHK(ensure(t, a->pe, u4 * bound, st));
    CHK(ensure(t, a->parent, u4 * bound, st));
    CHK(ensure(t, a->child, 8 * u4 * bound, st));
    CHK(ensure(t, a->leaf, bound + 4, st));  // read back as whole words by the export
    CHK(ensure(t, a->cmask, bound, st));
    CHK(ensure(t, a->nchild, u4 * bound, st));
    CHK(ensure(t, a->coff, u4 * (bound + 1), st));
    unsigned int *dc = bp<unsigned int>(t->counters);
    uint32_t *code = bp<uint32_t>(a->code), *ps = bp<uint32_t>(a->ps), *pe = bp<uint32_t>(a->pe);
    int *parent = bp<int>(a->parent), *child = bp<int>(a->child);
    uint8_t *leaf = bp<uint8_t>(a->leaf);
    uint32_t *scan = bp<uint32_t>(t->scan);
    KeySortWork ksw;
    ksw.keys_a = bp<uint32_t>(a->ks_a);
    ksw.keys_b = bp<uint32_t>(a->ks_b);
    ksw.vals = bp<uint32_t>(a->ks_v);
    ksw.hist = bp<uint32_t>(a->ks_h);
    ksw.off = ksw.hist + hw;
    ksw.scan = ksw.off + hw + 1;
    const KeyIndex ki{bp<uint32_t>(a->cstart), bp<uint32_t>(a->skey), Lf, cl};
    auto host_read = [&]() -> fmm_status {
        HIPCHK(hipEventRecord(t->ev_counters, st));
        HIPCHK(hipEventSynchronize(t->ev_counters));
        return FMM_OK;
    };
    HIPCHK(launch_keys(n, dtype, pos, c.box_lo, c.box_size, Lf, bp<uint32_t>(t->key10), nullptr, nullptr, dc, st));
    HIPCHK(launch_key_sort(n, Lf, bp<uint32_t>(t->key10), ksw, bp<uint32_t>(t->perm), bp<uint32_t>(a->skey), st));
    HIPCHK(launch_records(n, Lf, bp<uint32_t>(t->perm), bp<uint32_t>(t->key10), dtype, pos, c.box_lo, c.box_size,
                          bp<double4>(t->xyz64), st));
    HIPCHK(launch_key_starts(n, Lf, cl, bp<uint32_t>(a->skey), bp<uint32_t>(a->cstart), st));
    a->off[0] = 0;
    a->off[1] = 1;
    HIPCHK(ad_launch_root((uint32_t)n, code, ps, pe, parent, st));
    int l = 0;
    for (;; ++l) {
        const int64_t b0 = a->off[l], nb = a->off[l + 1] - a->off[l];
        HIPCHK(ad_launch_count(b0, nb, l, Lf, c.leaf_max, code, ps, pe, ki, leaf, bp<uint32_t>(a->nchild),
                               bp<uint8_t>(a->cmask), st));
        HIPCHK(launch_scan(nb, bp<uint32_t>(a->nchild), bp<uint32_t>(a->coff), scan, st));
        HIPCHK(ad_launch_children(b0, nb, l, Lf, a->off[l + 1], ki, bp<uint32_t>(a->coff),
                                  bp<uint8_t>(a->cmask), code, ps, pe, parent, child, st));
        HIPCHK(hipMemcpyAsync(a->hbuf, bp<uint32_t>(a->coff) + nb, u4, hipMemcpyDeviceToHost, st));
        if (l == 0) HIPCHK(hipMemcpyAsync(a->hbuf + 1, dc, u4, hipMemcpyDeviceToHost, st));
        CHK(host_read());
        if (l == 0 && a->hbuf[1] != 0)
            return fail(FMM_EDOMAIN, std::to_string(a->hbuf[1]) + " positions outside the root cube or not finite");
        const int64_t kids = a->hbuf[0];
        if (kids == 0) break;
        if (a->off[l + 1] + kids > bound) return fail(FMM_EDEVICE, "internal: box count over its bound");
        a->off[l + 2] = a->off[l + 1] + kids;
    }
    const int nlev = l + 1;
    const int64_t nbox = a->off[nlev];
    a->depth = l;
    a->nbox = nbox;
    a->nvbox = nlev > 2 ? nbox - a->off[2] : 0;
    if (!t->ops) CHK(build_ops(c.p, &t->ops));
    CHK(ensure(t, a->lev, u4 * nbox, st));
    CHK(ensure(t, a->col, 27 * u4 * nbox, st));
    CHK(ensure(t, a->vidx, (size_t)kOffsetsPerClass * u4 * std::max<int64_t>(a->nvbox, 1), st));
    CHK(ensure(t, a->offd, sizeof(int64_t) * (nlev + 1), st));
    const int64_t n27 = 27 * nbox;  // (box, direction) pairs of the list passes
    CHK(ensure(t, a->cnts, 3 * u4 * n27, st));
    CHK(ensure(t, a->s27, 3 * u4 * (n27 + 1), st));
    CHK(ensure(t, a->offs, 3 * u4 * (nbox + 1), st));
    CHK(ensure(t, t->scan, u4 * scan_scratch_words(std::max(3 * n27, n) + 1), st));
    scan = bp<uint32_t>(t->scan);
    CHK(ensure(t, a->is_head, u4 * n, st));
    CHK(ensure(t, a->head, u4 * n, st));
    CHK(ensure(t, a->hoff, u4 * (n + 1), st));
    const int ngrp = 8 * std::max(nlev - 2, 0);
    CHK(ensure(t, a->ccnt, u4 * std::max(ngrp, 1), st));
    int *lev = bp<int>(a->lev), *col = bp<int>(a->col), *vidx = bp<int>(a->vidx);
    uint32_t *nu = bp<uint32_t>(a->cnts), *nw = nu + n27, *nx = nw + n27;
    // the U, W and X counts (contiguous) in one scan: run k starts at k n27
    uint32_t *su = bp<uint32_t>(a->s27), *sw = su + n27, *sx = sw + n27;
    uint32_t *ou = bp<uint32_t>(a->offs), *ow = ou + nbox + 1, *ox = ow + nbox + 1;
    HIPCHK(hipMemcpyAsync(a->offd.p, a->off, sizeof(int64_t) * (nlev + 1), hipMemcpyHostToDevice, st));
    HIPCHK(ad_launch_structure(nbox, nlev, a->off, bp<int64_t>(a->offd), code, parent, child, lev, col,
                               t->ops->cls, vidx, st));
    HIPCHK(ad_launch_lists(nbox, 0, lev, code, parent, col, child, leaf, nu, nw, nx, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, st));
    HIPCHK(launch_scan(3 * n27, nu, su, scan, st));
    HIPCHK(ad_launch_box_offsets(nbox, su, ou, ow, ox, st));
    HIPCHK(launch_zero(bp<uint32_t>(a->is_head), n, st));
    HIPCHK(ad_launch_heads(nbox, leaf, ps, pe, bp<uint32_t>(a->is_head), bp<int>(a->head), st));
    HIPCHK(launch_scan(n, bp<uint32_t>(a->is_head), bp<uint32_t>(a->hoff), scan, st));
    if (ngrp) {
        HIPCHK(launch_zero(bp<uint32_t>(a->ccnt), ngrp, st));
        HIPCHK(ad_launch_class(a->off[2], a->nvbox, lev, code, bp<unsigned int>(a->ccnt), nullptr, nullptr,
                               nullptr, st));
        HIPCHK(hipMemcpyAsync(a->hbuf + 4, a->ccnt.p, u4 * ngrp, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(a->hbuf, ou + nbox, u4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(a->hbuf + 1, ow + nbox, u4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(a->hbuf + 2, ox + nbox, u4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(a->hbuf + 3, bp<uint32_t>(a->hoff) + n, u4, hipMemcpyDeviceToHost, st));
    CHK(host_read());
    for (int k = 0; k < 3; ++k) a->nlist[k] = a->hbuf[k];
    a->nleaf = a->hbuf[3];
    CHK(ensure(t, a->iu, u4 * std::max<int64_t>(a->nlist[0], 1), st));
    CHK(ensure(t, a->iw, u4 * std::max<int64_t>(a->nlist[1], 1), st));
    CHK(ensure(t, a->ix, u4 * std::max<int64_t>(a->nlist[2], 1), st));
    HIPCHK(ad_launch_lists(nbox, 1, lev, code, parent, col, child, leaf, nu, nw, nx, su, sw, sx, bp<int>(a->iu),
                           bp<int>(a->iw), bp<int>(a->ix), st));
    CHK(ensure(t, a->lbox, u4 * a->nleaf, st));
    CHK(ensure(t, a->lstart, u4 * (a->nleaf + 1), st));
    CHK(ensure(t, a->llev, a->nleaf, st));
    HIPCHK(launch_zero(dc + 3, 1, st));
    HIPCHK(ad_launch_leaflist(n, a->nleaf, bp<uint32_t>(a->is_head), bp<uint32_t>(a->hoff), bp<int>(a->head), ps,
                              bp<int>(a->lbox), bp<uint32_t>(a->lstart), bp<uint8_t>(a->llev), lev, dc + 3, st));
    HIPCHK(ad_launch_records(n, dtype, bp<uint32_t>(a->hoff), bp<int>(a->lbox), lev, code, bp<uint32_t>(t->perm),
                             pos, c.box_lo, c.box_size, bp<double4>(t->xyz64), st));
    // P2P work units: at most one per leaf plus one per 64 particles
    a->max_units = a->nleaf + n / 64;
    // (heaviest units first: one run of nleaf counts per weight class and
    // order, P2P over U and M2P over W, and one scan)
    CHK(ensure(t, a->ucnt, u4 * 2 * kAdUnitClasses * a->nleaf, st));
    CHK(ensure(t, a->uoff, u4 * (2 * kAdUnitClasses * a->nleaf + 1), st));
    CHK(ensure(t, a->units, sizeof(int2) * a->max_units, st));
    CHK(ensure(t, a->units_m, sizeof(int2) * a->max_units, st));
    HIPCHK(ad_launch_units(a->nleaf, 0, bp<uint32_t>(a->lstart), bp<int>(a->lbox), ou, ow, bp<int>(a->iu), ps, pe,
                           bp<uint32_t>(a->ucnt), nullptr, nullptr, nullptr, st));
    HIPCHK(launch_scan(2 * kAdUnitClasses * a->nleaf, bp<uint32_t>(a->ucnt), bp<uint32_t>(a->uoff), scan, st));
    HIPCHK(ad_launch_units(a->nleaf, 1, bp<uint32_t>(a->lstart), bp<int>(a->lbox), ou, ow, bp<int>(a->iu), ps, pe,
                           bp<uint32_t>(a->ucnt), bp<uint32_t>(a->uoff), bp<int2>(a->units), bp<int2>(a->units_m),
                           st));
    // M2L targets grouped by (level, class), tiles of 128 targets per block
    a->plan = AdM2LPlan{};
    int64_t at = 0;
    for (int g = 0; g < ngrp; ++g) {
        a->goff[g] = at;
        const int64_t cnt = a->hbuf[4 + g];
        if (cnt) {
            AdM2LGroup &e = a->plan.grp[a->plan.ngroups++];
            e.unit0 = a->plan.units;
            e.toff = at;
            e.count = cnt;
            e.cls = g % 8;
            e.lev = 2 + g / 8;
            a->plan.units += (cnt + 127) / 128;
        }
        at += cnt;
    }
    a->goff[ngrp] = at;
    // K-split so that the launch has about four blocks per compute unit
    a->plan.nsplit = a->plan.units ? (int)std::min<int64_t>(8, std::max<int64_t>(1, (4 * t->ncu + a->plan.units - 1) /
                                                                                         a->plan.units))
                                   : 1;
    if (at != a->nvbox) return fail(FMM_EDEVICE, "internal: M2L groups do not cover the boxes");
    if (ngrp) {
        CHK(ensure(t, a->tgt, u4 * a->nvbox, st));
        CHK(ensure(t, a->goffd, sizeof(int64_t) * (ngrp + 1), st));
        HIPCHK(hipMemcpyAsync(a->goffd.p, a->goff, sizeof(int64_t) * (ngrp + 1), hipMemcpyHostToDevice, st));
        HIPCHK(launch_zero(bp<uint32_t>(a->ccnt), ngrp, st));
        HIPCHK(ad_launch_class(a->off[2], a->nvbox, lev, code, nullptr, bp<int64_t>(a->goffd),
                               bp<unsigned int>(a->ccnt), bp<int>(a->tgt), st));
    }
    t->L = a->depth;
    t->nleaf = a->nleaf;
    t->max_count = -1;  // read by fmm_tree_info
    ++t->gen;           // a captured graph holds this tree's launch shapes
    return FMM_OK;
}

// Evaluation on an adaptive tree: gather, P2M at the leaves, M2M up to level
// 2, P2L over X (which writes every box's locals) and M2L over the V slots
// (added), L2L down, L2P and M2P over W at the leaves, P2P over U, all in
// FP64 except the mixed form's M2L (binary16 parts on the 16-bit matrix
// cores, its operands packed after P2L).  The stage events keep the uniform
// chain's numbering, with P2L and the operand pack in the place of the pack
// (stage 3) and M2P with L2P (stage 6).
// The adjoint runs the same launches on the weights with the transposed
// operators: P2M as L2P^T and the upward pass with L2L^T (the M buffer then
// holds the local adjoints), P2L as M2P^T and M2L^T over the same V slots
// (V is symmetric) into the L buffer, the downward pass with M2M^T, then
// L2P and M2P as P2M^T and P2L^T with their position derivatives (X and W
// are each other's transposes), and P2P on the weights (U is symmetric).
fmm_status run_adaptive(fmm_tree *t, const Work &w, const void *charges, bool adjoint, bool do_far, bool do_near,
                        hipStream_t st, const Combine *fuse = nullptr, bool *fused = nullptr) {
    const AdTree *a = t->ad;
    const int P = t->cfg.p, S = coef_stride(P);
    const Ops *o = t->ops;
    t->cur = (int)(t->ncalls % kTimeRing);
    if (t->xyz64.cap < sizeof(double4) * (size_t)t->n || a->lbox.cap < sizeof(int) * (size_t)a->nleaf)
        return fail(FMM_EDEVICE, "internal: adaptive tree buffers do not match");
    double4 *recs = bp<double4>(t->xyz64);
    const int *lbox = bp<int>(a->lbox), *lev = bp<int>(a->lev);
    const uint32_t *lstart = bp<uint32_t>(a->lstart), *code = bp<uint32_t>(a->code);
    const uint32_t *ps = bp<uint32_t>(a->ps), *pe = bp<uint32_t>(a->pe);
    const uint32_t *ou = bp<uint32_t>(a->offs), *ow = ou + a->nbox + 1, *ox = ow + a->nbox + 1;
    CHK(rec(t, 0, st));
    HIPCHK(launch_gather_q(t->n, t->dtype, true, bp<uint32_t>(t->perm), charges, recs, st));
    // the near field on the library's side stream beside the far field
    // (cfg.overlap_near), as in the uniform chain: P2P reads only the records
    // and writes its own buffer
    const bool far = do_far && a->depth >= 2;
    const bool side = do_near && far && t->cfg.overlap_near && !t->quiet;
    t->p2p_side[t->cur] = side;
    // the mixed form: FP32 pair arithmetic in P2P, FP32 terms in P2M, P2L,
    // L2P and M2P
    const bool f32 = t->cfg.precision == FMM_PREC_MIXED;
    auto p2p = [&](hipStream_t s2, const Combine *cf) -> hipError_t {
        return ad_launch_p2p(a->max_units, bp<uint32_t>(a->uoff) + kAdUnitClasses * a->nleaf, bp<int2>(a->units),
                             lbox, lstart, ou, bp<int>(a->iu), lev, code, ps, pe, recs, w.nearf, cf, f32, s2);
    };
    if (side) {
        if (!t->side) {
            HIPCHK(hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&t->ev_fork, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&t->ev_join, hipEventDisableTiming));
        }
        HIPCHK(hipEventRecord(t->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(t->side, t->ev_fork, 0));
        CHK(rec(t, kStages + 1, t->side));
        HIPCHK(p2p(t->side, nullptr));
        CHK(rec(t, kStages + 2, t->side));
        HIPCHK(hipEventRecord(t->ev_join, t->side));
    }
    CHK(rec(t, 1, st));
    if (far) {
        if (!o || !w.farf || !w.M[0] || !w.Lc[0] || w.m2lpart_bytes < ad_m2l_partial_bytes(a->plan, P))
            return fail(FMM_EDEVICE, "internal: no far-field buffers");
        double *M = (double *)w.M[0], *Lc = (double *)w.Lc[0];
        const bool half = m2l_half(t->cfg);
        if (half && (!w.pack[0] || !w.lmax)) return fail(FMM_EDEVICE, "internal: no binary16 operand buffers");
        HIPCHK(launch_zero((uint32_t *)(M + (size_t)a->nbox * S), 2 * S, st));  // the zero row
        const int adj = adjoint ? 1 : 0;
        const uint8_t *llev = bp<uint8_t>(a->llev);
        HIPCHK(ad_launch_p2m(P, a->nleaf, lbox, lstart, llev, adj, recs, M, f32, st));
        CHK(rec(t, 2, st));
        for (int l = a->depth - 1; l >= 2; --l)
            HIPCHK(ad_launch_m2m(P, a->off[l], a->off[l + 1] - a->off[l], bp<uint8_t>(a->leaf), bp<int>(a->child),
                                 adjoint ? o->aup64 : o->up64, M, st));
        CHK(rec(t, 3, st));
        HIPCHK(ad_launch_p2l(P, a->nbox, ox, bp<int>(a->ix), lev, code, ps, pe, adj, recs, Lc, f32, st));
        if (half) {  // the mixed form's operands: level maxima, scaled binary16 parts
            HIPCHK(launch_zero(w.lmax, kLevelSlots, st));
            HIPCHK(ad_launch_pack_h(P, a->off[2], a->nbox, lev, M, o->rho_inv, w.lmax, w.pack[0], st));
        }
        CHK(rec(t, 4, st));
        if (half)
            HIPCHK(ad_launch_m2l_h(P, a->plan, adjoint ? o->am2lh : o->m2lh, o->bf_part, o->cls, w.pack[0],
                                   bp<int>(a->vidx), a->off[2], bp<int>(a->tgt), a->nbox, w.lmax,
                                   adjoint ? o->aoscale : o->oscale, Lc, w.m2lpart, st));
        else
            HIPCHK(ad_launch_m2l(P, a->plan, adjoint ? o->am2l64 : o->m2l64, o->cls, M, bp<int>(a->vidx), a->off[2],
                                 bp<int>(a->tgt), a->nbox, Lc, w.m2lpart, st));
        CHK(rec(t, 5, st));
        for (int l = 3; l <= a->depth; ++l)
            HIPCHK(ad_launch_l2l(P, a->off[l], a->off[l + 1] - a->off[l], code, bp<int>(a->parent),
                                 adjoint ? o->adown64 : o->down64, Lc, st));
        CHK(rec(t, 6, st));
        HIPCHK(ad_launch_l2p(P, a->nleaf, lbox, lstart, llev, adj, recs, Lc, w.farf, f32, st));
        HIPCHK(ad_launch_m2p(P, a->max_units, bp<uint32_t>(a->uoff) + kAdUnitClasses * a->nleaf,
                             bp<int2>(a->units_m), adj, lbox, lstart, ow, bp<int>(a->iw), lev, code, recs, M, w.farf,
                             f32, st));
    } else {
        for (int s = 2; s <= 6; ++s) CHK(rec(t, s, st));
    }
    CHK(rec(t, 7, st));
    if (side) {
        HIPCHK(hipStreamWaitEvent(st, t->ev_join, 0));
    } else if (do_near) {  // last on the call's stream: it takes over the combine
        HIPCHK(p2p(st, fuse));
        if (fused) *fused = fuse != nullptr;
    } else {
        HIPCHK(launch_zero((uint32_t *)w.nearf, 8 * t->n, st));
    }
    CHK(rec(t, 8, st));
    return FMM_OK;
}

// ---------------------------------------------------------------- graphs
bool slot_matches(const fmm_tree *t, const GraphSlot &g, const void *const arg[5], int32_t flags) {
    if (!g.exec || g.gen != t->gen || g.L != t->L || g.n != t->n || g.flags != flags) return false;
    if (std::memcmp(&g.cfg, &t->cfg, sizeof(fmm_config)) != 0) return false;
    for (int i = 0; i < 5; ++i)
        if (g.arg[i] != arg[i]) return false;
    return true;
}

fmm_status drop_graph(GraphSlot &g) {
    if (!g.exec) return FMM_OK;
    // the previous graph may still run on the stream of its latest launch
    if (g.last) HIPCHK(hipStreamSynchronize(g.last));
    HIPCHK(hipGraphExecDestroy(g.exec));
    g.exec = nullptr;
    g.last = nullptr;
    return FMM_OK;
}

// Capture `chain` (the launches of one call, issued on the stream it is
// given) into `g`.  Capturing executes nothing.
template <typename Chain>
fmm_status capture_graph(fmm_tree *t, GraphSlot &g, const void *const arg[5], int32_t flags,
                         Chain chain) {
    CHK(drop_graph(g));
    if (!t->cap) HIPCHK(hipStreamCreateWithFlags(&t->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(t->cap, hipStreamCaptureModeThreadLocal));
    t->capturing = true;
    const fmm_status s = chain(t->cap);
    t->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(t->cap, &graph);
    if (s != FMM_OK) {
        if (e == hipSuccess && graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return fail(FMM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        g.exec = nullptr;
        return fail(FMM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    g.gen = t->gen;
    g.L = t->L;
    g.n = t->n;
    g.cfg = t->cfg;
    g.flags = flags;
    for (int i = 0; i < 5; ++i) g.arg[i] = arg[i];
    return FMM_OK;
}

fmm_status launch_graph(GraphSlot &g, hipStream_t st) {
    HIPCHK(hipGraphLaunch(g.exec, st));
    g.last = st;
    return FMM_OK;
}

fmm_status evaluate_chain(fmm_tree *t, const void *q, void *phi, void *vec, int32_t flags,
                          hipStream_t st, bool noalloc = false) {
    const int kind = flags & 3, part = flags & ~3;
    const bool do_far = part != FMM_PART_NEAR_ONLY, do_near = part != FMM_PART_FAR_ONLY;
    Work w;
    CHK(noalloc ? work_from_scratch(t, do_far, w) : work_from_tree(t, do_far, st, w));
    // the adaptive kernels leave their results in units of the root box
    const double inv_w = (t->ad ? 1.0 : (double)((int64_t)1 << t->L)) / t->cfg.box_size;
    const Combine c{(const uint32_t *)t->perm.p, (t->L >= 2 && do_far) ? w.farf : nullptr, inv_w, q, phi,
                    vec, kind, t->dtype};
    bool fused = false;
    CHK(t->ad ? run_adaptive(t, w, q, false, do_far, do_near, st, &c, &fused)
              : run_chain(t, w, q, false, do_far, do_near, st, &c, &fused));
    if (!fused) HIPCHK(launch_combine(t->n, w.nearf, c, st));
    CHK(rec(t, kStages, st));
    if (t->cfg.profile && !t->quiet) ++t->ncalls;
    return FMM_OK;
}

fmm_status backward_chain(fmm_tree *t, const void *q, const void *w, const void *field_fwd,
                          void *grad_q, void *grad_pos, hipStream_t st) {
    Work wk;
    CHK(work_from_tree(t, true, st, wk));
    CHK(t->ad ? run_adaptive(t, wk, w, true, true, true, st) : run_chain(t, wk, w, true, true, true, st));
    const double inv_w = (t->ad ? 1.0 : (double)((int64_t)1 << t->L)) / t->cfg.box_size;
    HIPCHK(launch_combine_grad(t->n, t->dtype, (const uint32_t *)t->perm.p, wk.nearf,
                               t->L >= 2 ? wk.farf : nullptr, inv_w, q, w, field_fwd, grad_q,
                               grad_pos, st));
    CHK(rec(t, kStages, st));
    if (t->cfg.profile) ++t->ncalls;
    return FMM_OK;
}

// P2P and M2L pair counts of a uniform tree
fmm_status uniform_counts(fmm_tree *t, fmm_tree_info_t *info) {
    CHK(ensure(t, t->pairs, sizeof(unsigned long long), t->stream));
    HIPCHK(launch_pair_count(t->L, (const uint32_t *)t->start.p, (unsigned long long *)t->pairs.p, t->stream));
    unsigned long long pairs = 0;
    HIPCHK(hipMemcpyAsync(&pairs, t->pairs.p, sizeof(pairs), hipMemcpyDeviceToHost, t->stream));
    HIPCHK(hipStreamSynchronize(t->stream));
    info->p2p_pairs = (int64_t)pairs - t->n;
    // M2L pairs: per axis the count factorises; sum over targets of
    // (children of in-domain parent neighbours) - (in-domain near boxes)
    int64_t m2l = 0;
    for (int l = 2; l <= t->L; ++l) {
        const int64_t n = (int64_t)1 << l, h = n / 2;
        int64_t sc = 0, sm = 0;
        for (int64_t x = 0; x < n; ++x) {
            const int64_t pp = x / 2;
            sc += 2 * ((pp - 1 >= 0) + 1 + (pp + 1 < h));
            sm += (x - 1 >= 0) + 1 + (x + 1 < n);
        }
        m2l += sc * sc * sc - sm * sm * sm;
    }
    info->m2l_pairs = m2l;
    return FMM_OK;
}

}  // namespace

extern "C" {

void fmm_config_default(fmm_config *c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->abi_version = FMM_ABI_VERSION;
    c->p = 8;
    c->leaf_max = 64;
    c->max_level = FMM_MAX_LEVEL;
    c->precision = FMM_PREC_MIXED;
    c->bf16_splits = 3;
    c->m2l_fp16 = 1;
    c->box_size = 1.0;
}

const char *fmm_status_string(fmm_status s) {
    switch (s) {
        case FMM_OK: return "ok";
        case FMM_EINVAL: return "invalid argument";
        case FMM_EDOMAIN: return "position outside the domain or not finite";
        case FMM_ENOMEM: return "out of device memory";
        case FMM_EDEVICE: return "HIP device error";
        case FMM_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *fmm_last_error_message(void) { return g_err.c_str(); }

fmm_status fmm_build_tree(const fmm_config *cfg, int64_t n, int32_t dtype, const void *pos,
                          void *stream, fmm_tree **out) {
    CHK(validate_cfg(cfg));
    if (n < 1) return fail(FMM_EINVAL, "n must be >= 1");
    if (n >= ((int64_t)1 << 31)) return fail(FMM_EINVAL, "n must be < 2^31");
    if (dtype != FMM_F32 && dtype != FMM_F64) return fail(FMM_EINVAL, "unknown dtype");
    if (!pos) return fail(FMM_EINVAL, "pos is NULL");
    if (!out) return fail(FMM_EINVAL, "out is NULL");
    hipStream_t st = (hipStream_t)stream;
    fmm_tree *t = *out;
    const bool fresh = (t == nullptr);
    // A tree is rebuilt in place only under the settings its operator tables,
    // particle records and buffers were made for: checked before anything
    // is allocated or launched, so that a rejected call leaves it untouched.
    if (!fresh) {
        const fmm_config &o = t->cfg;
        const bool mixed = cfg->precision == FMM_PREC_MIXED;
        if (o.p != cfg->p || o.precision != cfg->precision || t->dtype != dtype ||
            (mixed && (split_parts(o) != split_parts(*cfg) || !o.m2l_fp16 != !cfg->m2l_fp16)) ||
            !o.adaptive != !cfg->adaptive)
            return fail(FMM_EINVAL, "a tree is rebuilt only with the p, precision, M2L encoding "
                                    "(bf16_splits, m2l_fp16), tree kind and dtype it was created with");
        if (o.alloc != cfg->alloc || o.free != cfg->free || o.alloc_ctx != cfg->alloc_ctx)
            return fail(FMM_EINVAL, "a tree is rebuilt only with the allocator it was created with");
    }
    if (fresh) {
        t = new (std::nothrow) fmm_tree();
        if (!t) return fail(FMM_ENOMEM, "host allocation failed");
    }
    auto bail = [&](fmm_status s) {
        if (fresh) {
            fmm_tree_destroy(t);
            *out = nullptr;
        }
        return s;
    };
    t->cfg = *cfg;
    t->dtype = dtype;
    t->n = n;
    t->stream = st;
    t->al.fa = cfg->alloc;
    t->al.ff = cfg->free;
    t->al.ctx = cfg->alloc_ctx;
    if (hipGetDevice(&t->dev) != hipSuccess) return bail(fail(FMM_EDEVICE, "hipGetDevice failed"));
    if (hipDeviceGetAttribute(&t->ncu, hipDeviceAttributeMultiprocessorCount, t->dev) != hipSuccess ||
        t->ncu < 1)
        return bail(fail(FMM_EDEVICE, "cannot read the compute unit count"));
    if (!t->al.fa) ensure_pool(t->dev);
    if (!t->host_counters) {
        if (hipHostMalloc((void **)&t->host_counters, 4 * sizeof(unsigned int), hipHostMallocCoherent) !=
            hipSuccess)
            return bail(fail(FMM_EDEVICE, "hipHostMalloc failed"));
        if (hipHostGetDevicePointer((void **)&t->host_counters_dev, t->host_counters, 0) != hipSuccess)
            return bail(fail(FMM_EDEVICE, "hipHostGetDevicePointer failed"));
    }
    fmm_status s;
    // S1: smallest level whose fullest leaf holds <= leaf_max; the coarsest
    // candidate is the first level with 8^l * leaf_max >= n (fewer boxes
    // cannot hold n particles under the cap).  For the uniform inputs of the
    // method it is also the answer almost surely, so the sort at that level
    // is queued before the host has read the counters: the host waits only
    // for the counter copy, and queues a rebuild at a finer level in the rare
    // case that the candidate's fullest leaf is over the cap.
    int lev = 0;
    while (lev < cfg->max_level && ((int64_t)1 << (3 * lev)) * (int64_t)cfg->leaf_max < n) ++lev;
    if (!t->ev_counters && hipEventCreateWithFlags(&t->ev_counters, hipEventDisableTiming) != hipSuccess)
        return bail(fail(FMM_EDEVICE, "hipEventCreate failed"));
    if (cfg->adaptive) {
        if ((s = build_adaptive(t, n, dtype, pos, st)) != FMM_OK) return bail(s);
        *out = t;
        return FMM_OK;
    }
    const bool f64 = is_f64_form(t);
    if ((s = ensure(t, t->key10, sizeof(uint32_t) * n, st)) != FMM_OK) return bail(s);
    if ((s = ensure(t, t->rank, sizeof(uint32_t) * n, st)) != FMM_OK) return bail(s);
    if ((s = ensure(t, t->counters, 4 * sizeof(unsigned int), st)) != FMM_OK) return bail(s);
    if ((s = ensure(t, t->tmp, sizeof(uint32_t) * n, st)) != FMM_OK) return bail(s);
    if ((s = ensure(t, t->perm, sizeof(uint32_t) * n, st)) != FMM_OK) return bail(s);
    if (f64) {
        if ((s = ensure(t, t->xyz64, sizeof(double4) * n, st)) != FMM_OK) return bail(s);
    } else {
        if ((s = ensure(t, t->xyz32, sizeof(int4) * n, st)) != FMM_OK) return bail(s);
    }
    auto level_buffers = [&](int l) -> fmm_status {
        const size_t nb = (size_t)1 << (3 * l);
        fmm_status r;
        if ((r = ensure(t, t->cnt, sizeof(uint32_t) * nb, st)) != FMM_OK) return r;
        if ((r = ensure(t, t->start, sizeof(uint32_t) * (nb + 1), st)) != FMM_OK) return r;
        return ensure(t, t->scan, sizeof(uint32_t) * scan_scratch_words((int64_t)nb), st);
    };
    unsigned int *dc = (unsigned int *)t->counters.p;
    // leaf starts (scan of the counts) and the fullest leaf, and the two
    // build counters in the pinned host words (stored by the scan when it is
    // one kernel, else copied)
    auto read_counters = [&](int l) -> hipError_t {
        bool direct = false;
        hipError_t r = launch_scan_max((int64_t)1 << (3 * l), (const uint32_t *)t->cnt.p,
                                       (uint32_t *)t->start.p, (uint32_t *)t->scan.p, dc + 1, dc,
                                       t->host_counters_dev, &direct, st);
        if (r == hipSuccess && !direct)
            r = hipMemcpyAsync(t->host_counters, dc, 2 * sizeof(unsigned int), hipMemcpyDeviceToHost, st);
        if (r == hipSuccess) r = hipEventRecord(t->ev_counters, st);
        return r;
    };
    // placement and the in-leaf ordering (after read_counters at level l)
    auto sort_at = [&](int l) -> hipError_t {
        const uint32_t skip = l < cfg->max_level ? (uint32_t)cfg->leaf_max : UINT32_MAX;
        return launch_sort(n, l, skip, (const uint32_t *)t->key10.p, (const uint32_t *)t->rank.p,
                           (const uint32_t *)t->start.p, (uint32_t *)t->tmp.p, dtype, pos, cfg->box_lo,
                           cfg->box_size, (uint32_t *)t->perm.p, f64 ? nullptr : (int4 *)t->xyz32.p,
                           f64 ? (double4 *)t->xyz64.p : nullptr, st);
    };
    if ((s = level_buffers(lev)) != FMM_OK) return bail(s);
    hipError_t e = launch_keys(n, dtype, pos, cfg->box_lo, cfg->box_size, lev, (uint32_t *)t->key10.p,
                               (uint32_t *)t->cnt.p, (uint32_t *)t->rank.p, dc, st);
    if (e == hipSuccess) e = read_counters(lev);
    if (e == hipSuccess) e = sort_at(lev);
    if (e == hipSuccess) e = hipEventSynchronize(t->ev_counters);
    if (e != hipSuccess) return bail(fail(FMM_EDEVICE, std::string("tree build: ") + hipGetErrorString(e)));
    if (t->host_counters[0] != 0)
        return bail(fail(FMM_EDOMAIN, std::to_string(t->host_counters[0]) +
                                          " positions outside the root cube or not finite"));
    t->max_count = t->host_counters[1];
    if (t->max_count > cfg->leaf_max && lev < cfg->max_level) {
        do {
            ++lev;
            if ((s = level_buffers(lev)) != FMM_OK) return bail(s);
            e = launch_hist(n, (const uint32_t *)t->key10.p, lev, (uint32_t *)t->cnt.p,
                            (uint32_t *)t->rank.p, dc, st);
            if (e == hipSuccess) e = read_counters(lev);
            if (e == hipSuccess) e = hipEventSynchronize(t->ev_counters);
            if (e != hipSuccess) return bail(fail(FMM_EDEVICE, std::string("level selection: ") + hipGetErrorString(e)));
            t->max_count = t->host_counters[1];
        } while (t->max_count > cfg->leaf_max && lev < cfg->max_level);
        e = sort_at(lev);
        if (e != hipSuccess) return bail(fail(FMM_EDEVICE, std::string("sort: ") + hipGetErrorString(e)));
    }
    t->L = lev;
    t->nleaf = (int64_t)1 << (3 * lev);
    // translation tables of this p (made once per device and p): a tree with
    // a far field has them before its first evaluation
    if (lev >= 2 && !t->ops && (s = build_ops(cfg->p, &t->ops)) != FMM_OK) return bail(s);
    if (lev >= 2 && cfg->precision == FMM_PREC_FP64 && cfg->m2l_rotation && !t->ops->rot64 &&
        (s = build_rot_ops(cfg->p, t->ops)) != FMM_OK)
        return bail(s);
    *out = t;
    return FMM_OK;
}

fmm_status fmm_evaluate(fmm_tree *t, const void *q, void *phi, void *vec, int32_t flags,
                        void *stream) {
    if (!t || !q || !phi) return fail(FMM_EINVAL, "tree, q and phi are required");
    const int kind = flags & 3, part = flags & ~3;
    if (kind == 3 || (part != 0 && part != FMM_PART_NEAR_ONLY && part != FMM_PART_FAR_ONLY))
        return fail(FMM_EINVAL, "unknown flags");
    if (kind != FMM_VEC_NONE && !vec) return fail(FMM_EINVAL, "vec is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (!t->cfg.graph) return evaluate_chain(t, q, phi, vec, flags, st);
    const void *arg[5] = {q, phi, vec, nullptr, nullptr};
    if (slot_matches(t, t->gfwd, arg, flags)) return launch_graph(t->gfwd, st);
    CHK(evaluate_chain(t, q, phi, vec, flags, st));
    return capture_graph(t, t->gfwd, arg, flags, [&](hipStream_t cs) {
        return evaluate_chain(t, q, phi, vec, flags, cs);
    });
}

fmm_status fmm_evaluate_noalloc(fmm_tree *t, const void *q, void *phi, void *vec, int32_t flags,
                                void *stream) {
    if (!t || !q || !phi) return fail(FMM_EINVAL, "tree, q and phi are required");
    const int kind = flags & 3, part = flags & ~3;
    if (kind == 3 || (part != 0 && part != FMM_PART_NEAR_ONLY && part != FMM_PART_FAR_ONLY))
        return fail(FMM_EINVAL, "unknown flags");
    if (kind != FMM_VEC_NONE && !vec) return fail(FMM_EINVAL, "vec is NULL");
    if (t->L >= 2 && !t->ops) return fail(FMM_EINVAL, "the tree has no translation tables");
    // serial order, no events, no graph: nothing here creates a stream, an
    // event or a buffer
    t->quiet = true;
    const fmm_status s = evaluate_chain(t, q, phi, vec, flags, (hipStream_t)stream, true);
    t->quiet = false;
    return s;
}

fmm_status fmm_backward(fmm_tree *t, const void *q, const void *w, const void *field_fwd,
                        void *grad_q, void *grad_pos, void *stream) {
    if (!t || !q || !w) return fail(FMM_EINVAL, "tree, q and w are required");
    if (grad_pos && !field_fwd) return fail(FMM_EINVAL, "field_fwd is required for grad_pos");
    if (!grad_q && !grad_pos) return FMM_OK;
    hipStream_t st = (hipStream_t)stream;
    if (!t->cfg.graph) return backward_chain(t, q, w, field_fwd, grad_q, grad_pos, st);
    const void *arg[5] = {q, w, field_fwd, grad_q, grad_pos};
    if (slot_matches(t, t->gbwd, arg, 0)) return launch_graph(t->gbwd, st);
    CHK(backward_chain(t, q, w, field_fwd, grad_q, grad_pos, st));
    return capture_graph(t, t->gbwd, arg, 0, [&](hipStream_t cs) {
        return backward_chain(t, q, w, field_fwd, grad_q, grad_pos, cs);
    });
}

fmm_status fmm_tree_info(const fmm_tree *tc, fmm_tree_info_t *info) {
    if (!tc || !info) return fail(FMM_EINVAL, "tree and info are required");
    fmm_tree *t = const_cast<fmm_tree *>(tc);
    std::memset(info, 0, sizeof(*info));
    info->levels = t->L;
    info->p = t->cfg.p;
    info->n = t->n;
    info->n_leaves = t->nleaf;
    info->max_leaf_count = t->max_count;
    if (t->ad) {
        const AdTree *a = t->ad;
        CHK(ensure(t, t->pairs, 4 * sizeof(unsigned long long), t->stream));
        HIPCHK(launch_zero((uint32_t *)t->pairs.p, 8, t->stream));
        const uint32_t *ou = bp<uint32_t>(a->offs), *ow = ou + a->nbox + 1, *ox = ow + a->nbox + 1;
        HIPCHK(ad_launch_counts(a->nbox, a->off[std::min(a->depth + 1, 2)], bp<uint8_t>(a->leaf),
                                bp<uint32_t>(a->ps), bp<uint32_t>(a->pe), ou, bp<int>(a->iu), ow, ox,
                                bp<int>(a->ix), bp<int>(a->vidx), (unsigned long long *)t->pairs.p, t->stream));
        unsigned long long c[4] = {};
        unsigned int mx = 0;
        HIPCHK(hipMemcpyAsync(c, t->pairs.p, sizeof(c), hipMemcpyDeviceToHost, t->stream));
        HIPCHK(hipMemcpyAsync(&mx, (unsigned int *)t->counters.p + 3, sizeof(mx), hipMemcpyDeviceToHost,
                              t->stream));
        HIPCHK(hipStreamSynchronize(t->stream));
        info->max_leaf_count = mx;
        info->p2p_pairs = (int64_t)c[0] - t->n;
        info->m2l_pairs = (int64_t)c[1];
        info->m2p_evals = (int64_t)c[2];
        info->p2l_evals = (int64_t)c[3];
        info->n_boxes = a->nbox;
    } else {
        info->n_boxes = 0;
        for (int l = 0; l <= t->L; ++l) info->n_boxes += (int64_t)1 << (3 * l);
        CHK(uniform_counts(t, info));
    }
    size_t ws = 0;
    const Buf *bufs[] = {&t->key10, &t->rank, &t->cnt, &t->start, &t->tmp, &t->perm, &t->scan,
                         &t->counters, &t->xyz32, &t->xyz64, &t->nearf, &t->farf, &t->pairs, &t->m2lpart, &t->lmax};
    for (const Buf *b : bufs) ws += b->cap;
    for (int l = 0; l <= FMM_MAX_LEVEL; ++l) ws += t->M[l].cap + t->Lc[l].cap + t->pack[l].cap;
    if (t->ad)
        for (const Buf *b : t->ad->bufs()) ws += b->cap;
    info->workspace_bytes = ws;
    return FMM_OK;
}


fmm_status fmm_stage_times(const fmm_tree *t, double *ms, int32_t n_stages) {
    if (!t || !ms) return fail(FMM_EINVAL, "tree and ms are required");
    if (!t->cfg.profile || t->ncalls == 0) return fail(FMM_EINVAL, "profiling is off or nothing was recorded");
    const int ns = std::min<int>(n_stages, kStages);
    const int64_t nset = std::min<int64_t>(t->ncalls, kTimeRing);
    for (int i = 0; i < ns; ++i) ms[i] = 0.0;
    for (int64_t c = t->ncalls - nset; c < t->ncalls; ++c) {
        const int j = (int)(c % kTimeRing);
        for (int i = 0; i < ns; ++i) {
            if (!stage_on(t, i)) continue;
            float f = 0.f;
            if (i == 7 && t->p2p_side[j]) {  // P2P ran on the side stream
                HIPCHK(hipEventSynchronize(t->ev[j][kStages + 2]));
                HIPCHK(hipEventElapsedTime(&f, t->ev[j][kStages + 1], t->ev[j][kStages + 2]));
            } else {
                HIPCHK(hipEventSynchronize(t->ev[j][i + 1]));
                HIPCHK(hipEventElapsedTime(&f, t->ev[j][i], t->ev[j][i + 1]));
            }
            ms[i] += f;
        }
    }
    for (int i = 0; i < ns; ++i) ms[i] = stage_on(t, i) ? ms[i] / (double)nset : std::nan("");
    return FMM_OK;
}

fmm_status fmm_stage_times_reset(fmm_tree *t) {
    if (!t) return fail(FMM_EINVAL, "tree is NULL");
    t->ncalls = 0;
    return FMM_OK;
}

fmm_status fmm_tree_export(const fmm_tree *t, uint32_t *perm, uint32_t *leaf_start) {
    if (!t) return fail(FMM_EINVAL, "tree is NULL");
    if (perm) HIPCHK(hipMemcpyAsync(perm, t->perm.p, sizeof(uint32_t) * t->n, hipMemcpyDeviceToHost, t->stream));
    if (leaf_start)
        HIPCHK(hipMemcpyAsync(leaf_start, t->ad ? t->ad->lstart.p : t->start.p, sizeof(uint32_t) * (t->nleaf + 1),
                              hipMemcpyDeviceToHost, t->stream));
    HIPCHK(hipStreamSynchronize(t->stream));
    return FMM_OK;
}

fmm_status fmm_tree_export_adaptive(const fmm_tree *t, int64_t *sizes, int32_t *boxes, uint32_t *perm,
                                    int64_t *list_start, int32_t *items) {
    if (!t || !sizes) return fail(FMM_EINVAL, "tree and sizes are required");
    if (!t->ad) return fail(FMM_EINVAL, "not an adaptive tree");
    const AdTree *a = t->ad;
    const int64_t nbox = a->nbox;
    hipStream_t st = t->stream;
    auto get = [&](std::vector<uint32_t> &v, const void *src, size_t words) -> fmm_status {
        v.resize(std::max<size_t>(words, 1));
        if (words) HIPCHK(hipMemcpyAsync(v.data(), src, 4 * words, hipMemcpyDeviceToHost, st));
        return FMM_OK;
    };
    std::vector<uint32_t> vid;
    CHK(get(vid, a->vidx.p, (size_t)kOffsetsPerClass * a->nvbox));
    HIPCHK(hipStreamSynchronize(st));
    int64_t nv = 0;
    for (int64_t i = 0; i < kOffsetsPerClass * a->nvbox; ++i) nv += (int32_t)vid[i] >= 0;
    const int64_t box2 = nbox - a->nvbox;
    sizes[0] = nbox;
    sizes[1] = a->nlist[0];
    sizes[2] = nv;
    sizes[3] = a->nlist[1];
    sizes[4] = a->nlist[2];
    sizes[5] = a->depth;
    if (boxes) {
        std::vector<uint32_t> code, ps, pe, parent, lev, leaf;
        CHK(get(code, a->code.p, nbox));
        CHK(get(ps, a->ps.p, nbox));
        CHK(get(pe, a->pe.p, nbox));
        CHK(get(parent, a->parent.p, nbox));
        CHK(get(lev, a->lev.p, nbox));
        CHK(get(leaf, a->leaf.p, (nbox + 3) / 4));
        HIPCHK(hipStreamSynchronize(st));
        const uint8_t *lf = (const uint8_t *)leaf.data();
        for (int64_t b = 0; b < nbox; ++b) {
            int32_t *o = boxes + 8 * b;
            uint32_t xyz[3] = {0, 0, 0};
            for (int bit = 0; bit < 10; ++bit)
                for (int ax = 0; ax < 3; ++ax) xyz[ax] |= ((code[b] >> (3 * bit + ax)) & 1u) << bit;
            o[0] = (int32_t)lev[b];
            o[1] = (int32_t)xyz[0];
            o[2] = (int32_t)xyz[1];
            o[3] = (int32_t)xyz[2];
            o[4] = (int32_t)ps[b];
            o[5] = (int32_t)pe[b];
            o[6] = (int32_t)parent[b];
            o[7] = lf[b];
        }
    }
    if (perm) {
        HIPCHK(hipMemcpyAsync(perm, t->perm.p, sizeof(uint32_t) * t->n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (list_start || items) {
        std::vector<uint32_t> offs, iu, iw, ix;
        CHK(get(offs, a->offs.p, 3 * (nbox + 1)));
        CHK(get(iu, a->iu.p, a->nlist[0]));
        CHK(get(iw, a->iw.p, a->nlist[1]));
        CHK(get(ix, a->ix.p, a->nlist[2]));
        HIPCHK(hipStreamSynchronize(st));
        const uint32_t *ou = offs.data(), *ow = ou + nbox + 1, *ox = ow + nbox + 1;
        int64_t *su = list_start, *sv = su ? su + (nbox + 1) : nullptr, *sw = sv ? sv + (nbox + 1) : nullptr,
                *sx = sw ? sw + (nbox + 1) : nullptr;
        int32_t *it = items;
        for (int64_t b = 0; b <= nbox; ++b) {
            if (su) {
                su[b] = ou[b];
                sw[b] = ow[b];
                sx[b] = ox[b];
            }
        }
        if (it) {
            for (int64_t e = 0; e < a->nlist[0]; ++e) *it++ = (int32_t)iu[e];
        }
        int64_t at = 0;
        for (int64_t b = 0; b < nbox; ++b) {
            if (sv) sv[b] = at;
            if (b >= box2)
                for (int k = 0; k < kOffsetsPerClass; ++k) {
                    const int32_t v = (int32_t)vid[kOffsetsPerClass * (b - box2) + k];
                    if (v < 0) continue;
                    if (it) *it++ = v;
                    ++at;
                }
        }
        if (sv) sv[nbox] = at;
        if (it) {
            for (int64_t e = 0; e < a->nlist[1]; ++e) *it++ = (int32_t)iw[e];
            for (int64_t e = 0; e < a->nlist[2]; ++e) *it++ = (int32_t)ix[e];
        }
    }
    return FMM_OK;
}

void fmm_tree_destroy(fmm_tree *t) {
    if (!t) return;
    (void)drop_graph(t->gfwd);
    (void)drop_graph(t->gbwd);
    if (t->cap) (void)hipStreamDestroy(t->cap);
    hipStream_t st = t->stream;
    Buf *bufs[] = {&t->key10, &t->rank, &t->cnt, &t->start, &t->tmp, &t->perm, &t->scan,
                   &t->counters, &t->xyz32, &t->xyz64, &t->nearf, &t->farf, &t->pairs, &t->m2lpart, &t->lmax};
    for (Buf *b : bufs) release(t, *b, st);
    for (int l = 0; l <= FMM_MAX_LEVEL; ++l) {
        release(t, t->M[l], st);
        release(t, t->Lc[l], st);
        release(t, t->pack[l], st);
    }
    if (t->ad) {
        for (Buf *b : t->ad->bufs()) release(t, *b, st);
        if (t->ad->hbuf) (void)hipHostFree(t->ad->hbuf);
        delete t->ad;
    }
    if (t->ev_ready)
        for (int j = 0; j < kTimeRing; ++j)
            for (int i = 0; i < kEvents; ++i) (void)hipEventDestroy(t->ev[j][i]);
    if (t->side) {
        (void)hipStreamSynchronize(t->side);
        (void)hipStreamDestroy(t->side);
        (void)hipEventDestroy(t->ev_fork);
        (void)hipEventDestroy(t->ev_join);
    }
    if (t->ev_counters) (void)hipEventDestroy(t->ev_counters);
    if (t->host_counters) (void)hipHostFree(t->host_counters);
    delete t;
}

fmm_status fmm_operator_host(int32_t p, int32_t kind, int32_t index, double *out) {
    if (p < 1 || p > FMM_P_MAX || !out) return fail(FMM_EINVAL, "bad p or NULL output");
    if (kind == 0 || kind == 1) {
        if (index < 0 || index > 7) return fail(FMM_EINVAL, "octant must be in 0..7");
        if (kind == 0)
            op_m2m(p, index, out);
        else
            op_l2l(p, index, out);
        return FMM_OK;
    }
    if (kind == 2) {
        if (index < 0 || index >= 343) return fail(FMM_EINVAL, "offset index out of range");
        const int ox = index % 7 - 3, oy = (index / 7) % 7 - 3, oz = index / 49 - 3;
        if (std::max(std::abs(ox), std::max(std::abs(oy), std::abs(oz))) < 2)
            return fail(FMM_EINVAL, "M2L offsets need |o|_inf >= 2");
        op_m2l(p, ox, oy, oz, out);
        return FMM_OK;
    }
    if (kind == 3 || kind == 4) {
        if (index < 0 || index >= 343) return fail(FMM_EINVAL, "offset index out of range");
        const int ox = index % 7 - 3, oy = (index / 7) % 7 - 3, oz = index / 49 - 3;
        if (ox == 0 && oy == 0 && oz == 0) return fail(FMM_EINVAL, "the zero offset has no direction");
        std::vector<double> other((size_t)p * p * p * p);
        if (kind == 3)
            op_m2l_rotated(p, ox, oy, oz, out, other.data());
        else
            op_m2l_rotated(p, ox, oy, oz, other.data(), out);
        return FMM_OK;
    }
    return fail(FMM_EINVAL, "unknown operator kind");
}

}  // extern "C"

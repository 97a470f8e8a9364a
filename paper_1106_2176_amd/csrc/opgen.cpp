// opgen.cpp -- host generation of the translation operators (FP64).
//
// All operators act on real coefficient vectors (slot layout of cidx()):
//   multipole ("mu") vectors: mu = sum_j q_j rho(u_j), u = (x - c)/w, so the
//     complex multipole is M_n^m = mu_c + i mu_s, M_n^{-m} = (-1)^m conj(M_n^m);
//   local ("ell") vectors: the potential is phi(x) = (1/w) ell . rho(u); the
//     complex local coefficients are L_n^0 = ell_0, L_n^m = (ell_c - i ell_s)/2,
//     L_n^{-m} = (-1)^m conj(L_n^m), so that phi = (1/w) sum_{n,m} L_n^m R_n^m(u).
// Box widths scale out of every operator (1/r is homogeneous): with
// multipoles scaled by w^-n and locals by w^(n+1) the matrices do not depend
// on the level, so one set serves every level (the paper's precomputation of
// reusable terms, Sec. 2.1).
//   M2M child -> parent  M_n^m(P) = sum_{k,l} 2^(k-2n) R_{n-k}^{m-l}(s) M_k^l(child)
//   L2L parent -> child  L_j^v(c) = sum_{k,l} 2^(j-2k-1) R_{k-j}^{l-v}(s) L_k^l(P)
//   M2L source -> target L_k^l(t) = (-1)^k sum_{n,m} M_n^m(s) I_{n+k}^{m+l}(o)
// with s = 2b - 1 the child octant (child centre minus parent centre in units
// of half a child width) and o the integer offset (target minus source) in
// box widths.  These follow from the addition theorems
//   R_n^m(a + b) = sum R_k^l(a) R_{n-k}^{m-l}(b),
//   I_n^m(x - h) = sum R_k^l(h) I_{n+k}^{m+l}(x),
// of the harmonics defined in common.hpp; the irregular ones are
//   I_0^0 = 1/r,  I_m^m = -(2m-1) (x+iy)/r^2 I_{m-1}^{m-1},
//   I_{m+1}^m = (2m+1) z/r^2 I_m^m,
//   r^2 I_n^m = (2n-1) z I_{n-1}^m - (n-m-1)(n+m-1) I_{n-2}^m,
//   I_n^{-m} = (-1)^m conj(I_n^m).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "opgen.hpp"

namespace fmm {

using cplx = std::complex<double>;

namespace {

struct Harm {
    int N;  // degrees 0..N-1
    std::vector<cplx> v;
    explicit Harm(int n) : N(n), v((size_t)n * (2 * n - 1)) {}
    cplx &at(int n, int m) { return v[(size_t)n * (2 * N - 1) + (m + N - 1)]; }
    cplx get(int n, int m) const {
        if (n < 0 || n >= N || m > n || m < -n) return cplx(0.0, 0.0);
        return v[(size_t)n * (2 * N - 1) + (m + N - 1)];
    }
    void mirror() {
        for (int n = 0; n < N; ++n)
            for (int m = 1; m <= n; ++m) at(n, -m) = ((m & 1) ? -1.0 : 1.0) * std::conj(at(n, m));
    }
};

Harm regular(int N, double x, double y, double z) {
    Harm R(N);
    const double r2 = x * x + y * y + z * z;
    const cplx xib(x, -y);
    for (int m = 0; m < N; ++m) {
        R.at(m, m) = (m == 0) ? cplx(1.0, 0.0) : -(xib / (2.0 * m)) * R.at(m - 1, m - 1);
        if (m + 1 < N) R.at(m + 1, m) = z * R.at(m, m);
        for (int n = m + 2; n < N; ++n)
            R.at(n, m) = ((2.0 * n - 1.0) * z * R.at(n - 1, m) - r2 * R.at(n - 2, m)) /
                         double((n - m) * (n + m));
    }
    R.mirror();
    return R;
}

Harm irregular(int N, double x, double y, double z) {
    Harm I(N);
    const double r2 = x * x + y * y + z * z;
    const cplx xi(x, y);
    for (int m = 0; m < N; ++m) {
        I.at(m, m) = (m == 0) ? cplx(1.0 / std::sqrt(r2), 0.0)
                              : -(2.0 * m - 1.0) * (xi / r2) * I.at(m - 1, m - 1);
        if (m + 1 < N) I.at(m + 1, m) = (2.0 * m + 1.0) * z * I.at(m, m) / r2;
        for (int n = m + 2; n < N; ++n)
            I.at(n, m) = ((2.0 * n - 1.0) * z * I.at(n - 1, m) -
                          double((n - m - 1) * (n + m - 1)) * I.at(n - 2, m)) /
                         r2;
    }
    I.mirror();
    return I;
}

enum VecKind { MU = 0, ELL = 1 };

// Derivatives of the complex input X^{+l}, X^{-l} with respect to the real
// slots (c, s) of an input vector of the given kind.
struct InDeriv {
    cplx dp_c, dp_s, dm_c, dm_s;
};
InDeriv in_deriv(VecKind kind, int l) {
    const double sg = (l & 1) ? -1.0 : 1.0;
    if (kind == MU) return {cplx(1, 0), cplx(0, 1), cplx(sg, 0), cplx(0, -sg)};
    return {cplx(0.5, 0), cplx(0, -0.5), cplx(0.5 * sg, 0), cplx(0, 0.5 * sg)};
}

// Fill the real p^2 x p^2 matrix (row-major [out][in]) of the complex map
// Y_{n,m} = sum_{k,l} C(n,m,k,l) X_{k,l}, given input/output vector kinds.
template <class F>
void realify(int p, VecKind in_kind, VecKind out_kind, F C, double *out) {
    const int P2 = p * p;
    std::memset(out, 0, sizeof(double) * P2 * P2);
    for (int n = 0; n < p; ++n)
        for (int m = 0; m <= n; ++m)
            for (int k = 0; k < p; ++k)
                for (int l = 0; l <= k; ++l) {
                    // dY_{n,m}/dx for the input slots of (k, l)
                    cplx dyc, dys;
                    if (l == 0) {
                        dyc = C(n, m, k, 0);
                        dys = 0.0;
                    } else {
                        const InDeriv d = in_deriv(in_kind, l);
                        const cplx cp = C(n, m, k, l), cm = C(n, m, k, -l);
                        dyc = cp * d.dp_c + cm * d.dm_c;
                        dys = cp * d.dp_s + cm * d.dm_s;
                    }
                    const int ic = cidx(k, l), is = ic + 1;
                    if (m == 0) {
                        const int o = cidx(n, 0);
                        out[o * P2 + ic] = dyc.real();
                        if (l > 0) out[o * P2 + is] = dys.real();
                    } else {
                        const int oc = cidx(n, m), os = oc + 1;
                        const double f = (out_kind == MU) ? 1.0 : 2.0;
                        const double g = (out_kind == MU) ? 1.0 : -2.0;
                        out[oc * P2 + ic] = f * dyc.real();
                        out[os * P2 + ic] = g * dyc.imag();
                        if (l > 0) {
                            out[oc * P2 + is] = f * dys.real();
                            out[os * P2 + is] = g * dys.imag();
                        }
                    }
                }
}

}  // namespace

void op_m2m(int p, int octant, double *out) {
    const double s[3] = {double(2 * (octant & 1) - 1), double(2 * ((octant >> 1) & 1) - 1),
                         double(2 * ((octant >> 2) & 1) - 1)};
    const Harm R = regular(p, s[0], s[1], s[2]);
    realify(p, MU, MU,
            [&](int n, int m, int k, int l) -> cplx {
                if (k > n) return 0.0;
                return std::ldexp(1.0, k - 2 * n) * R.get(n - k, m - l);
            },
            out);
}

void op_l2l(int p, int octant, double *out) {
    const double s[3] = {double(2 * (octant & 1) - 1), double(2 * ((octant >> 1) & 1) - 1),
                         double(2 * ((octant >> 2) & 1) - 1)};
    const Harm R = regular(p, s[0], s[1], s[2]);
    realify(p, ELL, ELL,
            [&](int j, int v, int k, int l) -> cplx {
                if (k < j) return 0.0;
                return std::ldexp(1.0, j - 2 * k - 1) * R.get(k - j, l - v);
            },
            out);
}

void op_m2l_at(int p, double ox, double oy, double oz, double *out) {
    const Harm I = irregular(2 * p - 1, ox, oy, oz);
    realify(p, MU, ELL,
            [&](int k, int l, int n, int m) -> cplx {
                return ((k & 1) ? -1.0 : 1.0) * I.get(n + k, m + l);
            },
            out);
}

void op_m2l(int p, int ox, int oy, int oz, double *out) { op_m2l_at(p, ox, oy, oz, out); }

namespace {

// Gauss-Legendre nodes and weights on [-1, 1] (Newton's iteration on the
// Legendre polynomial from the Chebyshev-like initial guesses).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            if (n == 1) p0 = 1.0, p1 = z;
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

void op_rotation(int p, const double Q[9], double *out) {
    // Degree-n regular harmonics span a space that rotations map to itself,
    // so rho(Q u) = D rho(u) with D block diagonal by degree.  On the unit
    // sphere the real harmonics are orthogonal: with a quadrature exact for
    // the products (degree <= 2p - 2: Gauss-Legendre in cos(theta) times the
    // trapezoid rule in phi), D = (sum w rho(Q u) rho(u)^T) G^-1, G the
    // diagonal Gram matrix sum w rho(u) rho(u)^T.
    const int P2 = p * p, nt = p, nph = 2 * p;
    std::vector<double> zt, wt, a(P2), b(P2), G(P2, 0.0), B((size_t)P2 * P2, 0.0);
    gauss_legendre(nt, zt, wt);
    for (int i = 0; i < nt; ++i)
        for (int j = 0; j < nph; ++j) {
            const double ph = 2.0 * M_PI * j / nph, st = std::sqrt(1.0 - zt[i] * zt[i]);
            const double u[3] = {st * std::cos(ph), st * std::sin(ph), zt[i]};
            const double v[3] = {Q[0] * u[0] + Q[1] * u[1] + Q[2] * u[2], Q[3] * u[0] + Q[4] * u[1] + Q[5] * u[2],
                                 Q[6] * u[0] + Q[7] * u[1] + Q[8] * u[2]};
            regular_rho(p, u[0], u[1], u[2], a.data());
            regular_rho(p, v[0], v[1], v[2], b.data());
            const double wq = wt[i] * (2.0 * M_PI / nph);
            for (int n = 0; n < p; ++n)
                for (int r = n * n; r < (n + 1) * (n + 1); ++r) {
                    G[r] += wq * a[r] * a[r];
                    for (int c = n * n; c < (n + 1) * (n + 1); ++c) B[(size_t)r * P2 + c] += wq * b[r] * a[c];
                }
        }
    std::memset(out, 0, sizeof(double) * P2 * P2);
    for (int n = 0; n < p; ++n)
        for (int r = n * n; r < (n + 1) * (n + 1); ++r)
            for (int c = n * n; c < (n + 1) * (n + 1); ++c) out[(size_t)r * P2 + c] = B[(size_t)r * P2 + c] / G[c];
}

void op_m2l_rotated(int p, int ox, int oy, int oz, double *D, double *Tz) {
    // Q = R_y(-theta) R_z(-phi) takes the direction of o to +z
    const double r = std::sqrt(double(ox * ox + oy * oy + oz * oz));
    const double th = std::acos(oz / r), ph = std::atan2(double(oy), double(ox));
    const double ct = std::cos(th), st = std::sin(th), cp = std::cos(ph), sp = std::sin(ph);
    // R_z(-phi) = [[cp, sp, 0], [-sp, cp, 0], [0, 0, 1]]; R_y(-theta) = [[ct, 0, -st], [0, 1, 0], [st, 0, ct]]
    const double Q[9] = {ct * cp, ct * sp, -st, -sp, cp, 0.0, st * cp, st * sp, ct};
    op_rotation(p, Q, D);
    op_m2l_at(p, 0.0, 0.0, r, Tz);
}

// Round to nearest even bfloat16 (the top 16 bits of an IEEE binary32), then
// back to float.  Inputs here are finite.
static uint16_t bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}
static float bf16_float(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

void split_bf16(double x, int parts, uint16_t *out) {
    double r = x;
    for (int i = 0; i < parts; ++i) {
        out[i] = bf16_bits((float)r);
        r -= (double)bf16_float(out[i]);
    }
}

uint16_t f16_bits(double x) {
    const uint16_t sign = std::signbit(x) ? 0x8000u : 0u;
    const double a = std::fabs(x);
    if (a == 0.0) return sign;
    int e = 0;
    (void)std::frexp(a, &e);       // a in [2^(e-1), 2^e)
    const int E = std::max(e - 1, -14);  // binary16 exponent (subnormals: -14)
    const double ulp = std::ldexp(1.0, E - 10);
    double m = std::nearbyint(a / ulp);  // significand in ulps, ties to even
    int Eb = E;
    if (m >= 2048.0) {  // rounded up to the next binade
        m *= 0.5;
        Eb += 1;
    }
    if (m < 1024.0) return (uint16_t)(sign | (uint16_t)m);  // subnormal (E = -14)
    return (uint16_t)(sign | (uint16_t)((Eb + 15) << 10) | (uint16_t)(m - 1024.0));
}

double f16_value(uint16_t h) {
    const int ex = (h >> 10) & 31, man = h & 1023;
    const double v = ex == 0 ? std::ldexp((double)man, -24) : std::ldexp(1024.0 + man, ex - 25);
    return (h & 0x8000u) ? -v : v;
}

void split_f16(double x, uint16_t out[2]) {
    out[0] = f16_bits(x);
    out[1] = f16_bits(x - f16_value(out[0]));
}

void harmonic_scale(int p, double *rho) {
    std::vector<double> mx(p, 0.0), v((size_t)p * p);
    const double r = std::sqrt(3.0) / 2.0, golden = M_PI * (3.0 - std::sqrt(5.0));
    const int ns = 4096;  // directions on a Fibonacci sphere
    for (int i = 0; i < ns; ++i) {
        const double z = 1.0 - (2.0 * i + 1.0) / ns, s = std::sqrt(1.0 - z * z), ph = golden * i;
        regular_rho(p, r * s * std::cos(ph), r * s * std::sin(ph), r * z, v.data());
        for (int n = 0; n < p; ++n)
            for (int c = n * n; c < (n + 1) * (n + 1); ++c) mx[n] = std::max(mx[n], std::fabs(v[c]));
    }
    for (int n = 0; n < p; ++n) rho[n] = std::ldexp(1.0, (int)std::lround(std::log2(mx[n])));
}

}  // namespace fmm

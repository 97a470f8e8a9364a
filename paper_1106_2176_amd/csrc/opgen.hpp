// opgen.hpp -- host generation of translation operators (see opgen.cpp).
#pragma once
#include <stdint.h>

#include "common.hpp"

namespace fmm {

// Real p^2 x p^2 matrices, row-major [out][in], FP64.
void op_m2m(int p, int octant, double *out);  // child octant -> parent
void op_l2l(int p, int octant, double *out);  // parent -> child octant
void op_m2l(int p, int ox, int oy, int oz, double *out);  // source -> target, o = target - source
void op_m2l_at(int p, double ox, double oy, double oz, double *out);  // any offset, |o| > 0
// rho(Q u) = D rho(u) for the rotation Q (row-major 3 x 3): D block diagonal
// by degree
void op_rotation(int p, const double Q[9], double *D);
// M2L of offset o by rotation: the rotation D that takes o's direction to +z
// and the M2L matrix Tz of the offset (0, 0, |o|), so that
// op_m2l(o) = D^T Tz D (Tz couples only coefficients of equal order and
// equal cosine/sine kind)
void op_m2l_rotated(int p, int ox, int oy, int oz, double *D, double *Tz);

// x = b0 + b1 + ... (+ residual): successive round-to-nearest-even bfloat16
// parts of x (each the bf16 rounding of the remaining residual).
void split_bf16(double x, int parts, uint16_t *out);

// IEEE binary16 bits of x rounded to nearest even (subnormals kept; |x| must
// stay below 65520), and the value of such bits.
uint16_t f16_bits(double x);
double f16_value(uint16_t h);
// x = h0 + h1 (+ residual): h0 the binary16 rounding of x, h1 that of x - h0.
void split_f16(double x, uint16_t out[2]);

// Power-of-two size of the degree-n regular harmonics over a box, rho[n] for
// n < p: the largest |real or imaginary part of R_n^m(u)| over sampled u with
// |u| = sqrt(3)/2 (the corner distance of a unit box), rounded to the
// nearest power of two.  A multipole vector divided by rho and a local vector
// multiplied by it have entries of the size of the box's charge and of the
// potential, degree by degree; the M2L matrices scaled on both sides,
// rho_n T_nj rho_j, then have entries of comparable size.
void harmonic_scale(int p, double *rho);

}  // namespace fmm

// opgen.hpp -- host generation of translation operators (see opgen.cpp).
#pragma once
#include <stdint.h>

#include "common.hpp"

namespace fmm {

// Real p^2 x p^2 matrices, row-major [out][in], FP64.
void op_m2m(int p, int octant, double *out);  // child octant -> parent
void op_l2l(int p, int octant, double *out);  // parent -> child octant
void op_m2l(int p, int ox, int oy, int oz, double *out);  // source -> target, o = target - source

// x = b0 + b1 + ... (+ residual): successive round-to-nearest-even bfloat16
// parts of x (each the bf16 rounding of the remaining residual).
void split_bf16(double x, int parts, uint16_t *out);

}  // namespace fmm

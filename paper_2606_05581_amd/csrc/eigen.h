// Timing record of the eigen step's dense products (eigen.hip).
#pragma once
#include "msk_internal.h"

namespace msk {

// Summed kernel time and algorithmic flops of the eigen step's dense
// products, by precision (FP32: the products with C; FP64: the basis
// products and the final Rayleigh quotients).
struct EigGemmTimes {
  int64_t fp32_products = 0, fp64_products = 0;
  double fp32_ms = 0, fp32_flops = 0, fp64_ms = 0, fp64_flops = 0;
};

}  // namespace msk

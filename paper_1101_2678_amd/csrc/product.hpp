// product.hpp -- launchers of the product-and-argmax construction
// (Section III-A): every unvisited city draws its own uniform and the largest
// product choice * r wins.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aco_state.hpp"

namespace aco {

// The m tours of iteration `iter` with the product rule.
hipError_t launch_construct_product(const Colony& c, uint32_t iter, hipStream_t s);
// `count` independent selections: rows count x ld floats (ld = n rounded up
// to 64, zero padding), feasible count x n bytes, u count x n floats.
hipError_t launch_test_product_select(int n, int count, const float* rows,
                                      const uint8_t* feasible, const float* u, int32_t* out,
                                      hipStream_t s);

// Philox throughput probe: `waves` wavefronts each compute 640 Philox blocks
// (ten per lane) per step for `steps` steps; sink holds waves * 64 words.
hipError_t launch_probe_philox(int waves, int steps, uint32_t seed, uint32_t* sink,
                               hipStream_t s);

}  // namespace aco

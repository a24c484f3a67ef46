// nn.hpp -- nearest-neighbour candidate lists (Section II, the candidate-list
// variant of tour construction): device tables and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "aco_state.hpp"

namespace aco {

constexpr int kMaxNn = 64;  // one candidate per lane of a wavefront

// Candidate tables of one colony, carved out of a workspace of their own.
//   nn    list length, 1 <= nn <= min(64, n - 1)
//   kp    row pitch (entries) of both tables: nn rounded up to 32
//   nnl   n x kp uint16: row i holds the nn cities j != i with the smallest
//         d_ij, ordered by (d_ij, j); padding entries are 0
//   cand  n x kp uint64: (nnl[i][r] << 32) | bits(choice[i][nnl[i][r]]),
//         rebuilt from choice before every construction; padding 0
struct NnTables {
    int32_t nn, kp;
    uint16_t* nnl;
    uint64_t* cand;
};

inline int nn_pitch(int nn) { return (nn + 31) & ~31; }

// Device bytes of the two tables (each 256-byte aligned).
size_t nn_table_bytes(int n, int nn);
NnTables nn_carve(char* base, int n, int nn);

// Builds the lists from the colony's distance matrix (one workgroup per row).
hipError_t launch_nn_lists(const Colony& c, const NnTables& t, hipStream_t s);
// Rebuilds the packed candidate table from the current choice matrix, then
// constructs the m tours of iteration `iter` with the candidate-list rule.
hipError_t launch_construct_nn(const Colony& c, const NnTables& t, uint32_t iter, hipStream_t s);

// C_nn (nearest-neighbour tour from city 0, ties to the lowest index), tau0
// = fl32(m / C_nn) and the best-so-far reset, written to the colony.  Uses
// the successor table as scratch for 32-entry neighbour lists, so it must run
// before the first construction.
hipError_t launch_nn_tour(const Colony& c, hipStream_t s);

}  // namespace aco

// Renormalisation step of spin-adapted operators (dmrg_su2_product in
// include/dmrg.h): the blocks of a coupled product [A^k1 x B^k2]^k.
#pragma once
#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "common.h"
#include "dmrg.h"

namespace dmrg {

struct Su2Product {
  struct Block {
    int out, in;     // coupled sectors (bra, ket)
    int64_t offset;  // element offset of the block in the output data
    int ja, jb;      // blocks of A and B
    int ra, ca, rb, cb;
    double scale;
  };
  std::vector<Block> blocks;
  int64_t size = 0;
};

// The output blocks (host only; A and B need only their sector arrays).
Su2Product su2_product_plan(const dmrg_su2_window& w, const dmrg_su2_operator& a, const dmrg_su2_operator& b,
                            int tk1, int tk2, int tk, int parity_b);

// Writes every block's data (device); synchronises the stream.
void su2_product_run(const Su2Product& p, const dmrg_su2_operator& a, const dmrg_su2_operator& b, double* data,
                     hipStream_t s);

// The projection onto the kept multiplets (dmrg_su2_rotate): output blocks
// (g', g) with their offsets, and per output the input blocks it sums.
struct Su2Rotation {
  struct Out {
    int g2, g;
    int64_t offset;
    std::vector<int> blocks;
  };
  std::vector<Out> outs;
  int64_t size = 0;
};
Su2Rotation su2_rotation_plan(const dmrg_su2_basis& basis, int n_blocks, const int32_t* out_sector,
                              const int32_t* in_sector);
// Writes the rotated blocks (device); synchronises the stream.
void su2_rotation_run(const Su2Rotation& r, const dmrg_su2_basis& basis, const int32_t* out_sector,
                      const int32_t* in_sector, const int64_t* offset, const double* data, double* out,
                      hipStream_t s);

}  // namespace dmrg

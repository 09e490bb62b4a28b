// Internal declarations shared by the HIP sources of libgnk (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gnk.h"

namespace gnk {

// Launch-shape parameters of the Cauchy pair kernel, picked per problem size.
struct CauchyPlan {
  int tpb = 256;      // threads per block (4 wavefronts)
  int tpt = 1;        // target nodes per lane
  int splits = 1;     // number of source ranges (grid.y); partial sums reduced in order
  int64_t chunk = 0;  // sources per split (multiple of 16: four wave quarters of 4)
};

// align: the split length is a multiple of it (16 for FP64; 256 for the mixed
// kernel, whose four wavefronts each take whole 64-node source tiles)
CauchyPlan plan_cauchy(int64_t N, int ncols, int num_cu, int align = 16);

// Source records: rec[j*(ncols+1)] = eta_j, rec[j*(ncols+1) + 1 + r] = w_j,r.
// S_part[(g*ncols + r)*N + i] = sum_{j in split g, j != i} w_j,r / (eta_i - eta_j)
hipError_t launch_cauchy_fp64(const double2* rec, int64_t N, int ncols, const CauchyPlan& plan,
                              double2* S_part, hipStream_t st);

// Mixed-precision Cauchy sum: FP32 for far 64-node source tiles, FP64 otherwise.
struct MixedArgs {
  const double2* rec;          // FP64 records (as launch_cauchy_fp64)
  const float2* rec32;         // FP32 records: tile-local eta offsets and weights
  const double4* src_bounds;   // per 64-node tile {cx, cy, r, 0}
  const double4* tgt_bounds;   // per target tile of 64*tpt nodes {cx, cy, r, 0}
  double far2;                 // (1 + theta)^2: far when |c_t - c_s|^2 > far2 (r_t + r_s)^2
};
hipError_t launch_tile_bounds(const double2* rec, int64_t N, int ncols, int tile, double4* out, hipStream_t st);
hipError_t launch_records32(const double2* rec, const double4* src_bounds, int64_t N, int ncols, float2* rec32,
                            hipStream_t st);
hipError_t launch_cauchy_mixed(const MixedArgs& m, int64_t N, int ncols, const CauchyPlan& plan, double2* S_part,
                               hipStream_t st);

// y_k += sign * L x_k for every component k and column r (circulant blocks of Sec. 3.3).
hipError_t launch_circulant(const double* x, double* y, int64_t m1, int64_t n, int nrhs, double sign,
                            const double2* twiddle, hipStream_t st);
hipError_t launch_twiddles(double2* tw, int64_t n, hipStream_t st);
bool circulant_uses_fft(int64_t n);

}  // namespace gnk

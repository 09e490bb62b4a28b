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
  int tpb = 256;      // threads per block; one target node per thread
  int splits = 1;     // number of source ranges (grid.y); partial sums reduced in order
  int64_t chunk = 0;  // sources per split (even)
};

CauchyPlan plan_cauchy(int64_t N, int nrhs, int num_cu);

// S_part[(g*nrhs + r)*N + i] = sum_{j in split g, j != i} W[j*nrhs + r] / (eta_i - eta_j)
hipError_t launch_cauchy_fp64(const double2* eta, const double2* W, int64_t N, int nrhs,
                              const CauchyPlan& plan, double2* S_part, hipStream_t st);

// y_k += sign * L x_k for every component k and column r (circulant blocks of Sec. 3.3).
hipError_t launch_circulant(const double* x, double* y, int64_t m1, int64_t n, int nrhs, double sign,
                            const double2* twiddle, hipStream_t st);
hipError_t launch_twiddles(double2* tw, int64_t n, hipStream_t st);
bool circulant_uses_fft(int64_t n);

}  // namespace gnk

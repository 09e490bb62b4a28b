// Internal declarations shared by the HIP sources of libgnk (not part of the ABI).
//
// Every solve works on a batch of domains (one domain for the single-domain
// entry points). Domain d has N_d = m1_d * n_d nodes and ncols_d real columns;
// column (d, r) is a vector of length N_d stored at a flat offset. The device
// keeps one DomDev per domain and one ColDev per column.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gnk.h"

namespace gnk {

struct DomDev {
  // boundary data (caller-owned)
  const double2* eta;
  const double2* etap;
  const double2* etapp;
  const double2* A;
  const double2* Ap;
  // per-node workspace
  double2* rho;      // eta' / A
  double* dB;        // diag(B1)
  double* dD;        // diag(D1)
  double* e;         // vector e of the adjoint equation
  // Cauchy-sum workspace: records rec[j*stride + f], f = 0: eta_j, f = 1 + q: weight column q
  double2* rec;
  float2* rec32;     // FP32 records (tile-local eta offsets, weights)
  double2* parts;    // partial sums [splits][wcols][N]
  double4* sb;       // bounds of the 64-node source tiles {cx, cy, r, 0}
  double4* tb;       // bounds of the 64*tpt-node target tiles
  double far2;       // mixed precision: far when |c_t - c_s|^2 > far2 (r_t + r_s)^2
  int N, n, m1;
  int ncols;         // real columns of the domain
  int c0;            // first global column index
  int splits;        // source splits
  int chunk;         // sources per split
  int c;             // +1 bounded, -1 unbounded
};

struct ColDev {
  int d;             // domain
  int r;             // column within the domain
  int64_t off;       // offset of the column in flat vectors
};

// Cauchy sums S = E w for every domain of the batch and every weight column
// (wcols_d = lead + data * ncols_d: an optional leading column, then the
// domain's data columns):
//   parts_d[(g*wcols_d + q)*N_d + i] = sum_{j in split g, j != i} w_jq / (eta_i - eta_j)
// items: int4 {d, target tile, split, first weight column}; `width` columns per
// item (8, 4, 2 or 1), one workgroup per item. mixed: FP32 for far 64-node
// source tiles (rec32, sb, tb). active: optional per global column mask; an
// item whose data columns are all inactive is skipped.
hipError_t launch_pairs(const DomDev* doms, const int4* items, int nitems, int width, int tpt, int lead, int data,
                        bool mixed, const int* active, hipStream_t st);

// bounding circles of the tiles of `tile` nodes of every domain (source tiles
// of 64 nodes into sb, target tiles into tb)
hipError_t launch_tile_bounds(const DomDev* doms, int ndom, int maxN, int tile, bool target, hipStream_t st);
// FP32 records from the FP64 records of every domain
hipError_t launch_records32(const DomDev* doms, int ndom, int maxN, int lead, int data, hipStream_t st);

// y_k += sign * L x_k for a list of length-n vectors at the given flat offsets
// (the circulant blocks of Sec. 3.3); twiddle: the table for this n.
hipError_t launch_circulant(const double* x, double* y, const int64_t* offs, int nvec, int64_t n, double sign,
                            const double2* twiddle, hipStream_t st);
hipError_t launch_twiddles(double2* tw, int64_t n, hipStream_t st);
bool circulant_uses_fft(int64_t n);

}  // namespace gnk

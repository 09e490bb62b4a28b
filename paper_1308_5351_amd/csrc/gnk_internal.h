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

// Source tiles of the FP64 single-column far form: records hold eta and b
// relative to the centre of the node's tile of this size.
#ifndef GNK_FAR_TILE_LOG2
#define GNK_FAR_TILE_LOG2 8
#endif
constexpr int kFarTileLog2 = GNK_FAR_TILE_LOG2;
constexpr int kFarTile = 1 << kFarTileLog2;

// FP64 source records (double2 fields): a head {eta, u = -2 eta', (|eta'|^2, 0)}
// (eta' = eta - centre of the node's far-form tile), then wcols weights w_q,
// then wcols products b_q = w_q conj(eta')
constexpr int kRecHead = 3;
__host__ __device__ constexpr int rec_stride(int wcols) { return kRecHead + 2 * wcols; }
// FP32 records of mixed products: {v, (|v|^2, 0), w.., b..} (float2 fields;
// v the offset from the node's 64-node tile centre in units of its radius)
__host__ __device__ constexpr int rec32_stride(int wcols) { return 2 + 2 * wcols; }
// FP32 sources of the matrix-core far tiles, per block of 8 weight columns and
// 64-node source tile: 9 fields (v, then w of the block's columns 0..7, zero
// past the last column), each 64 float2 (one per node), so that a wave reads
// every field of a tile in one coalesced load
constexpr int kFar32Fields = 9;
__host__ __device__ constexpr int64_t far32_size(int N, int wcols) {
  return (int64_t)((wcols + 7) / 8) * ((N + 63) / 64) * kFar32Fields * 64;
}

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
  double* bu;        // (2 pi/n) N(t_i, t_i), the diagonal limit (e:N-tt)
  // Cauchy-sum workspace: records rec[j*stride + f], f = 0: eta_j, f = 1 + q: weight column q
  double2* rec;
  float2* rec32;     // FP32 records (tile-local eta offsets over the tile radius, |v|^2, weights, b = w conj(v))
  float2* far32;     // FP32 far-tile sources [8-column block][64-node tile][field][node] (see far32_size)
  double2* parts;    // partial sums [splits][wcols][N]
  double4* sb;       // bounds of the 64-node source tiles {cx, cy, r, 0}
  double4* sbf;      // bounds of the FP64 far-form source tiles (kFarTile nodes)
  double4* tb;       // bounds of the 64*tpt-node target tiles
  const double2* tz; // targets other than the nodes (Cauchy integral at interior
                     // points), or null: the targets are the nodes themselves
  int Nt;            // number of those targets
  double far2;       // mixed precision: far when |c_t - c_s|^2 > far2 (r_t + r_s)^2
  double far2d;      // FP64 far form: far when |c_t - c_s|^2 > far2d (r_t + r_s)^2
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
// ext: the single domain's targets are doms[0].tz (FP64 only)
hipError_t launch_pairs(const DomDev* doms, const int4* items, int nitems, int width, int tpt, int lead, int data,
                        bool mixed, bool ext, const int* active, hipStream_t st);
// resident workgroups per CU of the pair-kernel variant (width columns, tpt, mixed)
int pairs_blocks_per_cu(int width, int tpt, bool mixed);

// bounding circles of the tiles of `tile` nodes of every domain (source tiles
// of 64 nodes into sb, target tiles into tb)
// which: 0 source tiles (sb), 1 target tiles (tb), 2 far-form source tiles (sbf),
// 3 target tiles of the separate targets tz (tb)
hipError_t launch_tile_bounds(const DomDev* doms, int ndom, int maxN, int tile, int which, hipStream_t st);
hipError_t launch_node_tile_bounds(const DomDev* doms, int ndom, int maxN, int tpt, hipStream_t st);
// Treecode (csrc/tree.hip): boxes of kLeaf << l consecutive nodes at level l
constexpr int kLeaf = 256;
constexpr int kTreeMaxP = 48;
// bounding circles of the boxes of every level (at out + level_off[l]): level
// 0 holds the leaves in slot order (perm: slot -> leaf, invp: leaf -> slot),
// box b of level l the slots [b 2^l, (b + 1) 2^l); leafbox: the leaves'
// bounding boxes; bbox and rbits: scratch of one entry per box
hipError_t launch_box_bounds(const double2* eta, int N, const int* level_off, const int* level_nb, int levels,
                             const double4* leafbox, const int* perm, const int* invp, double4* bbox,
                             unsigned long long* rbits, double4* out, hipStream_t st);
// bounding boxes {xmin, xmax, ymin, ymax} of the leaves (kLeaf consecutive nodes)
hipError_t launch_leaf_boxes(const double2* eta, int N, int nleaf, double4* leafbox, hipStream_t st);
// multipole moments (p per box) of record weight field wo: leaves directly,
// then every level from its children; level_off/level_nb: host arrays
hipError_t launch_tree_moments(const double2* rec, int stride, int wo, int N, const double4* bounds, const int* perm,
                               const int* level_off, const int* level_nb, int levels, int p, double2* mom,
                               hipStream_t st);
// far boxes by their moments, near 64-node blocks directly, for weight column
// col of doms[0]; seg: per target tile, 4 splits + 1 bounds into list
hipError_t launch_tree_eval(const DomDev* doms, int tiles, int tpt, const int* seg, const int* list,
                            const double4* bounds, const double2* mom, int p, int splits, int col, int wcols,
                            const int* active, int lead, bool ext, hipStream_t st);
// FP32 records from the FP64 records of every domain; threads: the largest
// N_d * (weight columns rounded up to a multiple of 8) over the domains
hipError_t launch_records32(const DomDev* doms, int ndom, int64_t threads, int lead, int data, hipStream_t st);

// One block length of a circulant product: nvec length-n vectors at the flat
// offsets offs; tw the twiddle table of n (or the direct product's column).
struct CircClass {
  const int64_t* offs;
  int nvec;
  int64_t n;
  const double2* tw;
};
// y_k += sign * L x_k for every vector of every class (the circulant blocks of
// Sec. 3.3); all power-of-two lengths in one launch.
hipError_t launch_circulant(const double* x, double* y, const CircClass* cls, int ncls, double sign, hipStream_t st);
hipError_t launch_twiddles(double2* tw, int64_t n, hipStream_t st);
bool circulant_uses_fft(int64_t n);

// Geometric derivatives of s = sum_t c_t u_t^T Op_t v_t (Op_t = f_B or fC).
// Terms are grouped by their vector v; z = i c_t (f_B) or c_t (fC).
struct GeomTerm {
  const double* u;
  double2 z;
};
struct GeomGroup {
  const double* v;
  int t0, t1;        // terms [t0, t1) of the group
};
// source records {eta, b V_g (G), b, a U_g (G), a P} with nw = 2G + 2 weights
hipError_t launch_geom_weights(const double2* eta, const double2* etap, const double2* A, int N,
                               const GeomTerm* terms, const GeomGroup* groups, int G, int nw, double2* rec,
                               double2* Ut, double2* P, hipStream_t st);
// first- and second-order Cauchy sums of the nw weights, per source split
hipError_t launch_cauchy12(const double2* rec, int nwpad, int N, int nw, int chunk, int splits, double2* parts,
                           hipStream_t st);
int geom_width(int nw);
// gradients with respect to eta, eta', A (any output may be null)
hipError_t launch_geom_epilogue(const double2* etap, const double2* A, int N, int n, const GeomGroup* groups, int G,
                                const double2* Ut, const double2* P, const double2* parts, int nw, int splits,
                                double2* g_eta, double2* g_etap, double2* g_A, hipStream_t st);

// Fourier boundary curves eta_j(t) = sum_k c_{j,k} e^{i sgn k t} at t_p = 2 pi p/n
// (coef: m1 x nk, component-major) and the chain rule back to the coefficients
hipError_t launch_fourier_curve(const double2* coef, int m1, int n, int kmin, int nk, int sgn, double2* eta,
                                double2* etap, double2* etapp, hipStream_t st);
hipError_t launch_fourier_vjp(const double2* g_eta, const double2* g_etap, const double2* g_etapp, int m1, int n,
                              int kmin, int nk, int sgn, double2* g_coef, hipStream_t st);

}  // namespace gnk

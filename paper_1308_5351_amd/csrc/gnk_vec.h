// Device-side state of the restarted GMRES (one entry per right-hand side).
#pragma once

#include "gnk_internal.h"

namespace gnk {

constexpr int kMaxRestart = 256;
constexpr int kMaxChunk = 2048;   // elements per block of the Gram-Schmidt kernels
// component sums per chunk: a chunk of at most kMaxChunk entries meets at most
// (kMaxChunk - 1) / n + 2 components, n >= 2
constexpr int kMaxMeanSlots = (kMaxChunk - 1) / 2 + 2;

struct GmresState {
  double* bnorm;        // ||b_r||
  double* true_relres;  // ||b - A x|| / ||b|| at the last cycle start
  double* relres;       // Givens residual estimate
  double* invbeta;      // 1 / ||r|| at the cycle start (normalisation of V_0)
  double* H;            // Hessenberg matrices, (restart+1) x restart, column-major, per column r
  double* cs;           // Givens cosines  [r][kMaxRestart]
  double* sn;           // Givens sines    [r][kMaxRestart]
  double* g;            // rotated rhs     [r][kMaxRestart+1]
  double* y;            // back-substitution result [r][kMaxRestart]
  int* active;          // column still iterating in this cycle
  int* converged;       // column met tol at the last true-residual check
  int* kdim;            // Krylov dimension reached in this cycle
  int* inner_it;        // total Arnoldi steps
  int* live;            // number of active columns (single int)
  int* step;            // current Arnoldi step l of the cycle (single int; see k_gs_finish)
  int* done;            // columns whose step has closed (single int)
  int ldh;              // restart + 1
  int hstride;          // ldh * restart
};

}  // namespace gnk

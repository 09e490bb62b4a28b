// Per-node kernels around the Cauchy sum (preparation of source weights,
// operator epilogues, validation) and the kernels of the device-resident
// restarted GMRES (classical Gram-Schmidt with one re-orthogonalisation,
// Givens rotations, back substitution). All reductions run in a fixed order,
// so repeated runs are bitwise identical.
// Included by solver.hip (one translation unit with the host driver).
#pragma once
#include "gnk_vec.h"

namespace gnk {

namespace {

constexpr int kT = 256;   // threads per block of the vector kernels

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // wave reduction by shuffles, then across the waves of the block through LDS
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int k = 0; k < nw; ++k) s += sh[k];
  return s;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ bool finite2(double2 v) { return isfinite(v.x) && isfinite(v.y); }

}  // namespace

// ---------------------------------------------------------------- validation
__global__ void k_validate(const double2* eta, const double2* etap, const double2* A, const double2* etapp,
                           const double2* Ap, int N, int need_etap_nonzero, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int f = 0;
  const double2 a = A[i];
  const double2 e = eta[i], ep = etap[i];
  if (!finite2(a) || !finite2(e) || !finite2(ep)) f |= 1;
  if (a.x == 0.0 && a.y == 0.0) f |= 2;
  if (etapp && !finite2(etapp[i])) f |= 1;
  if (Ap && !finite2(Ap[i])) f |= 1;
  if (need_etap_nonzero && ep.x == 0.0 && ep.y == 0.0) f |= 4;
  if (f) atomicOr(flags, f);
}

__global__ void k_check_finite(const double* x, int64_t n, int* flags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) atomicOr(flags, 1);
}

// ------------------------------------------------------------ per-node setup
// rho = eta' / A  (the weight factor of eqs. (e:hD-bt), (e:(I-B)x))
__global__ void k_rho(const double2* etap, const double2* A, double2* rho, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double2 p = etap[i], a = A[i];
  const double d = a.x * a.x + a.y * a.y;
  rho[i] = make_double2((p.x * a.x + p.y * a.y) / d, (p.y * a.x - p.x * a.y) / d);
}

// reduce the split partial sums of column col of a Cauchy launch with ncols columns
__device__ __forceinline__ double2 reduce_parts(const double2* part, int splits, int ncols, int col, int N, int i) {
  double2 s = make_double2(0.0, 0.0);
  for (int g = 0; g < splits; ++g) {
    const double2 v = part[((size_t)g * ncols + col) * N + i];
    s.x += v.x;
    s.y += v.y;
  }
  return s;
}

// From S = E(eta'/A):  dB = diag(B1) = -(2/n) Im(A S),  dD = diag(D1) = -(2/n) Re(A S)
// (eqs. (e:(I-B)x), (e:hD-bt) with x = 1).
__global__ void k_diag_fbie(const double2* part, int splits, int ncols, const double2* A, int N, double two_n,
                            double* dB, double* dD) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double2 s = reduce_parts(part, splits, ncols, 0, N, i);
  const double2 a = A[i];
  const double re = a.x * s.x - a.y * s.y, im = a.x * s.y + a.y * s.x;
  dB[i] = -two_n * im;
  dD[i] = -two_n * re;
}

// From S = E eta':  e = 1 - c - (2/n) Im(S) + (2/n) Im(eta''/eta' - A'/A)   (eq. (e:bve))
__global__ void k_evec(const double2* part, int splits, const double2* etap, const double2* etapp, const double2* A,
                       const double2* Ap, int N, double two_n, double c, double* e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double2 s = reduce_parts(part, splits, 1, 0, N, i);
  const double2 p = etap[i], pp = etapp[i], a = A[i], ap = Ap[i];
  const double dp = p.x * p.x + p.y * p.y, da = a.x * a.x + a.y * a.y;
  const double im1 = (pp.y * p.x - pp.x * p.y) / dp;   // Im(eta''/eta')
  const double im2 = (ap.y * a.x - ap.x * a.y) / da;   // Im(A'/A)
  e[i] = 1.0 - c - two_n * s.y + two_n * (im1 - im2);
}

// ----------------------------------------------- source weights and means
// Source records for the Cauchy kernel: rec[j*stride] = eta_j,
// rec[j*stride + 1 + col0 + r] = C_j * v_j for column r (block (k, r) covers
// component k of column r), with
//   v = x * scale[r]                 (optional; written back to xout)
//   mean[r*m1 + k] = (1/n) sum_p v_{k n + p}   (optional)
// If lead_one, record field 1 is C_j itself (x == 1) and data columns start
// at col0 = 1.
__global__ __launch_bounds__(kT) void k_weights(const double2* __restrict__ eta, const double2* __restrict__ C,
                                                const double* __restrict__ x, const double* __restrict__ scale,
                                                const int* __restrict__ active, double* __restrict__ xout,
                                                double2* __restrict__ rec, int N, int n, int m1, int stride,
                                                int col0, int lead_one, double* __restrict__ mean) {
  __shared__ double sh[kT / 64];
  const int k = blockIdx.x, r = blockIdx.y;
  if (active && !active[r]) return;
  const double s = scale ? scale[r] : 1.0;
  const double* xr = x + (size_t)r * N + (size_t)k * n;
  double acc = 0.0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const int j = k * n + p;
    const double v = xr[p] * s;
    if (xout) xout[(size_t)r * N + j] = v;
    const double2 c = C[j];
    double2* rj = rec + (size_t)j * stride;
    rj[1 + col0 + r] = make_double2(c.x * v, c.y * v);
    if (r == 0) {
      rj[0] = eta[j];
      if (lead_one) rj[1] = c;
    }
    acc += v;
  }
  if (mean) {
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) mean[(size_t)r * m1 + k] = t / (double)n;
  }
}

// records from eta and column-major complex weights w (N x ncols)
__global__ void k_pack_records(const double2* __restrict__ eta, const double2* __restrict__ w, int N, int ncols,
                               double2* __restrict__ rec) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double2* rj = rec + (size_t)j * (ncols + 1);
  rj[0] = eta[j];
  for (int r = 0; r < ncols; ++r) rj[1 + r] = w[(size_t)r * N + j];
}

// Operator epilogue, for column r (grid.y) of x (N x nrhs), S from column (col0 + r):
//   y = a0 x + dsign dg x + cI Im(Cout S) + cR Re(Cout S) + mean[r][k(i)]
__global__ void k_epilogue(const double2* __restrict__ part, int splits, int ncols, int col0,
                           const double* __restrict__ x, const double2* __restrict__ Cout,
                           const double* __restrict__ dg, double a0, double dsign, double cI, double cR,
                           const double* __restrict__ mean, int n, int m1, const int* __restrict__ active,
                           double* __restrict__ y, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  if (active && !active[r]) return;
  const double2 s = reduce_parts(part, splits, ncols, col0 + r, N, i);
  const double2 c = Cout[i];
  const double re = c.x * s.x - c.y * s.y, im = c.x * s.y + c.y * s.x;
  const double xv = x[(size_t)r * N + i];
  double v = a0 * xv + cI * im + cR * re;
  if (dg) v += dsign * dg[i] * xv;
  if (mean) v += mean[(size_t)r * m1 + i / n];
  y[(size_t)r * N + i] = v;
}

// S[r*N + i] = sum over the splits of the partial Cauchy sums (fixed order)
__global__ void k_reduce_parts(const double2* __restrict__ part, int splits, int ncols, int N, double2* __restrict__ S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  S[(size_t)r * N + i] = reduce_parts(part, splits, ncols, r, N, i);
}

// out[r] = ||x_r||_2, one block per column, fixed-order reduction
__global__ __launch_bounds__(kT) void k_col_norms(const double* __restrict__ x, int N, double* __restrict__ out) {
  __shared__ double sh[kT / 64];
  const int r = blockIdx.x;
  const double* xr = x + (size_t)r * N;
  double acc = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) acc = __builtin_fma(xr[i], xr[i], acc);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[r] = sqrt(t);
}

// y = a x + b y  (elementwise over len)
__global__ void k_axpby(double a, const double* x, double b, double* y, int64_t len) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < len) y[i] = a * x[i] + b * y[i];
}

// ------------------------------------------------------------------ GMRES
// V holds the Krylov vectors: V_l column r at V + ((size_t)l*nrhs + r)*N.

// Dots of the block's chunk of w_r with V_0..V_{nvec-1}: wavefront q takes
// vectors l = q, q+4, ...; each lane sums its strided elements and the wave
// reduces by shuffles. partial[(r*nblk + blk)*ldp + l].
__device__ __forceinline__ void chunk_dots(const double* __restrict__ V, int nvec, const double* __restrict__ w,
                                           int i0, int i1, int N, int nrhs, int r, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int l = wv; l < nvec; l += nw) {
    const double* vl = V + ((size_t)l * nrhs + r) * N;
    double acc = 0.0;
    for (int i = i0 + lane; i < i1; i += 64) acc = __builtin_fma(vl[i], w[i - i0], acc);
    acc = wave_sum(acc);
    if (lane == 0) out[l] = acc;
  }
}

__global__ __launch_bounds__(kT) void k_gs_dot(const double* __restrict__ V, int nvec, const double* __restrict__ w,
                                               int N, int nrhs, int per_blk, const int* __restrict__ active,
                                               double* __restrict__ partial, int ldp) {
  const int r = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  if (!active[r]) return;
  const int i0 = blk * per_blk, i1 = min(N, i0 + per_blk);
  chunk_dots(V, nvec, w + (size_t)r * N + i0, i0, i1, N, nrhs, r, partial + ((size_t)r * nblk + blk) * ldp);
}

// h_l = sum over blocks of pin (fixed order); w -= sum_l h_l V_l on this
// block's chunk; H[:, col] (+)= h (block 0); then pout = the chunk's dots of the
// updated w with V_0..V_{nvec-1} (do_dots) or its squared norm (entry 0).
__global__ __launch_bounds__(kT) void k_gs_update(const double* __restrict__ V, int nvec, double* __restrict__ w,
                                                  int N, int nrhs, int per_blk, const int* __restrict__ active,
                                                  const double* __restrict__ pin, double* __restrict__ pout, int ldp,
                                                  double* __restrict__ H, int ldh, int hstride, int col,
                                                  int accumulate_h, int do_dots) {
  __shared__ double h[kMaxRestart + 1];
  __shared__ double sw[kMaxChunk];
  __shared__ double sh[kT / 64];
  const int r = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  if (!active[r]) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int l = wv; l < nvec; l += nw) {
    double acc = 0.0;
    for (int b = lane; b < nblk; b += 64) acc += pin[((size_t)r * nblk + b) * ldp + l];
    acc = wave_sum(acc);
    if (lane == 0) h[l] = acc;
  }
  __syncthreads();
  if (blk == 0) {
    double* Hr = H + (size_t)r * hstride + (size_t)col * ldh;
    for (int l = threadIdx.x; l < nvec; l += blockDim.x) Hr[l] = accumulate_h ? Hr[l] + h[l] : h[l];
  }
  const int i0 = blk * per_blk, i1 = min(N, i0 + per_blk);
  double* wr = w + (size_t)r * N;
  double nrm = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double v = wr[i];
    for (int l = 0; l < nvec; ++l) v = __builtin_fma(-h[l], V[((size_t)l * nrhs + r) * N + i], v);
    wr[i] = v;
    sw[i - i0] = v;
    nrm = __builtin_fma(v, v, nrm);
  }
  double* out = pout + ((size_t)r * nblk + blk) * ldp;
  if (do_dots) {
    __syncthreads();
    chunk_dots(V, nvec, sw, i0, i1, N, nrhs, r, out);
  } else {
    const double t = block_sum(nrm, sh);
    if (threadIdx.x == 0) out[0] = t;
  }
}

// partial norms^2 of columns of x (grid (nblk, nrhs)); entry (r*nblk + blk)*ldp
__global__ __launch_bounds__(kT) void k_norm_partial(const double* __restrict__ x, int N, int per_blk,
                                                     double* __restrict__ partial, int ldp) {
  __shared__ double sh[kT / 64];
  const int r = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  const int i0 = blk * per_blk, i1 = min(N, i0 + per_blk);
  const double* xr = x + (size_t)r * N;
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) acc = __builtin_fma(xr[i], xr[i], acc);
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[((size_t)r * nblk + blk) * ldp] = s;
}

// r = b - Ax (in place into ax) and partial ||r||^2
__global__ __launch_bounds__(kT) void k_residual(const double* __restrict__ b, double* __restrict__ ax, int N,
                                                 int per_blk, double* __restrict__ partial, int ldp) {
  __shared__ double sh[kT / 64];
  const int r = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  const int i0 = blk * per_blk, i1 = min(N, i0 + per_blk);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const size_t idx = (size_t)r * N + i;
    const double v = b[idx] - ax[idx];
    ax[idx] = v;
    acc = __builtin_fma(v, v, acc);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[((size_t)r * nblk + blk) * ldp] = s;
}

// One thread per column: ||b|| from partials.
__global__ void k_bnorm(const double* partial, int nblk, int ldp, int nrhs, GmresState st) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[((size_t)r * nblk + b) * ldp];
  st.bnorm[r] = sqrt(s);
}

// Start of a restart cycle, one thread per column: beta0 = ||r|| from the
// partials, true relative residual, convergence test, g = beta0 e_1.
__global__ void k_cycle_start(const double* partial, int nblk, int ldp, int nrhs, double tol, GmresState st) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0) *st.live = 0;
  __syncthreads();
  if (r >= nrhs) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[((size_t)r * nblk + b) * ldp];
  const double beta = sqrt(s);
  const double bn = st.bnorm[r];
  const double rel = bn > 0.0 ? beta / bn : 0.0;
  st.true_relres[r] = rel;
  st.relres[r] = rel;
  st.kdim[r] = 0;
  double* g = st.g + (size_t)r * (kMaxRestart + 1);
  if (bn == 0.0 || rel <= tol || beta == 0.0) {
    st.converged[r] = 1;
    st.active[r] = 0;
    st.invbeta[r] = 0.0;
    g[0] = 0.0;
  } else {
    st.converged[r] = 0;
    st.active[r] = 1;
    st.invbeta[r] = 1.0 / beta;
    g[0] = beta;
    atomicAdd(st.live, 1);
  }
}

// End of Arnoldi step `col`; one 64-lane block per column r: beta = ||w||
// from the partials, H(col+1, col) = beta, Givens rotations applied in LDS,
// residual estimate, stop test for this cycle.
__global__ __launch_bounds__(64) void k_arnoldi_finish(const double* partial, int nblk, int ldp, int col,
                                                       int restart, double tol, GmresState st) {
  __shared__ double hc[kMaxRestart + 2];
  __shared__ double cs_[kMaxRestart + 1];
  __shared__ double sn_[kMaxRestart + 1];
  const int r = blockIdx.x, lane = threadIdx.x;
  if (!st.active[r]) return;
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += partial[((size_t)r * nblk + b) * ldp];
  s = wave_sum(s);
  const double beta = sqrt(s);
  double* Hc = st.H + (size_t)r * st.hstride + (size_t)col * st.ldh;
  double* cs = st.cs + (size_t)r * kMaxRestart;
  double* sn = st.sn + (size_t)r * kMaxRestart;
  for (int k = lane; k <= col; k += 64) {
    hc[k] = Hc[k];
    if (k < col) {
      cs_[k] = cs[k];
      sn_[k] = sn[k];
    }
  }
  __syncthreads();
  if (lane == 0) {
    hc[col + 1] = beta;
    for (int k = 0; k < col; ++k) {
      const double t = cs_[k] * hc[k] + sn_[k] * hc[k + 1];
      hc[k + 1] = -sn_[k] * hc[k] + cs_[k] * hc[k + 1];
      hc[k] = t;
    }
    const double a = hc[col];
    const double den = hypot(a, beta);
    double c = 1.0, sv = 0.0;
    if (den > 0.0) { c = a / den; sv = beta / den; }
    cs[col] = c;
    sn[col] = sv;
    hc[col] = den;
    hc[col + 1] = 0.0;
    double* g = st.g + (size_t)r * (kMaxRestart + 1);
    const double gc = g[col];
    g[col + 1] = -sv * gc;
    g[col] = c * gc;
    const double est = fabs(sv * gc) / st.bnorm[r];
    st.relres[r] = est;
    st.kdim[r] = col + 1;
    st.inner_it[r] += 1;
    const bool stop = (est <= tol) || (beta == 0.0) || (col + 1 >= restart) || (den == 0.0);
    if (stop) {
      st.active[r] = 0;
      atomicSub(st.live, 1);
    } else {
      st.invbeta[r] = 1.0 / beta;
    }
  }
  __syncthreads();
  for (int k = lane; k <= col + 1; k += 64) Hc[k] = hc[k];
}

// Back substitution H y = g (upper triangular kdim x kdim after the Givens
// rotations); one 64-lane block per column, each row sum split over lanes.
__global__ __launch_bounds__(64) void k_backsolve(GmresState st) {
  __shared__ double ys[kMaxRestart];
  const int r = blockIdx.x, lane = threadIdx.x;
  const int k = st.converged[r] ? 0 : st.kdim[r];
  const double* Hr = st.H + (size_t)r * st.hstride;
  const double* g = st.g + (size_t)r * (kMaxRestart + 1);
  for (int l = k - 1; l >= 0; --l) {
    double s = 0.0;
    for (int q = l + 1 + lane; q < k; q += 64) s = __builtin_fma(Hr[(size_t)q * st.ldh + l], ys[q], s);
    s = wave_sum(s);
    if (lane == 0) {
      const double d = Hr[(size_t)l * st.ldh + l];
      ys[l] = d != 0.0 ? (g[l] - s) / d : 0.0;
    }
    __syncthreads();
  }
  double* y = st.y + (size_t)r * kMaxRestart;
  for (int l = lane; l < kMaxRestart; l += 64) y[l] = l < k ? ys[l] : 0.0;
}

// x_r += sum_{l < kdim_r} y_l V_l,r
__global__ void k_xupdate(const double* __restrict__ V, double* __restrict__ x, int N, int nrhs, GmresState st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  const int k = st.converged[r] ? 0 : st.kdim[r];
  if (k == 0) return;
  const double* y = st.y + (size_t)r * kMaxRestart;
  double v = x[(size_t)r * N + i];
  for (int l = 0; l < k; ++l) v = __builtin_fma(y[l], V[((size_t)l * nrhs + r) * N + i], v);
  x[(size_t)r * N + i] = v;
}

// inner_it counters etc. to zero
__global__ void k_gmres_init(int nrhs, GmresState st) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  st.inner_it[r] = 0;
  st.relres[r] = 1.0;
  st.true_relres[r] = 1.0;
  st.converged[r] = 0;
  st.active[r] = 0;
  st.kdim[r] = 0;
}

}  // namespace gnk

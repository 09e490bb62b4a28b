// Circulant blocks of the discretised singular operator M (paper Sec. 3.3):
//   (Lhat x) restricted to component k = L x_k,
//   L_pq = (-1)^(p-q) (1/n) cot((p-q) pi / n) (p != q), L_pp = 0.
// L is circulant, so L x_k = ifft(fft(b) .* fft(x_k)) (eq. (e:L-bs)) with b its
// first column; fft(b)_k equals 2 i k / n for the signed frequency |k| < n/2
// and 0 at k = n/2, so the symbol is applied in closed form.
//
// gfx950 mapping: one workgroup per PAIR of real length-n columns (two
// components, or two right-hand sides): because L is a real matrix,
// L (x_a + i x_b) = L x_a + i L x_b, so one complex FFT carries two real
// columns with no post-processing. The transform runs in LDS:
// a radix-2 decimation-in-frequency pass (natural order in, bit-reversed out),
// the symbol multiply in bit-reversed order, then a decimation-in-time inverse
// pass (bit-reversed in, natural out), so no permutation pass is needed.
// Global traffic is one read of x and one read-modify-write of y per element.
// The vectors are given as a list of flat offsets, so one launch covers every
// component of every column (and of every domain with this n).
// Powers of two up to 4096 use the FFT; other even n use a direct O(n^2)
// circulant product with the closed-form first column.
#include "gnk_internal.h"

namespace gnk {

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftMaxN = 4096;

__global__ void k_twiddles(double2* tw, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n / 2) {
    double s, c;
    sincospi(-2.0 * (double)k / (double)n, &s, &c);
    tw[k] = make_double2(c, s);   // exp(-2 pi i k / n)
  }
}

// first column of L for the direct fallback: b_d = (-1)^d (1/n) cot(d pi / n), b_0 = 0
__global__ void k_circ_column(double* b, int n) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d < n) {
    double v = 0.0;
    if (d != 0) {
      double s, c;
      sincospi((double)d / (double)n, &s, &c);
      v = ((d & 1) ? -1.0 : 1.0) * (c / s) / (double)n;
    }
    b[d] = v;
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {   // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// vectors: offs[v] is the flat offset of length-n vector v; block b takes v = 2b, 2b+1
__global__ __launch_bounds__(kFftThreads) void k_circulant_fft(const double* __restrict__ x, double* __restrict__ y,
                                                               const int64_t* __restrict__ offs, int n, int logn,
                                                               int V, double sign, const double2* __restrict__ tw) {
  extern __shared__ double2 z[];
  const int va = 2 * blockIdx.x;
  const int vb = va + 1;
  const bool hasb = vb < V;
  const int64_t oa = offs[va];
  const int64_t ob = hasb ? offs[vb] : 0;
  const double* xa = x + oa;
  const double* xb = x + ob;
  for (int p = threadIdx.x; p < n; p += blockDim.x) z[p] = make_double2(xa[p], hasb ? xb[p] : 0.0);

  const int half = n >> 1;
  // forward DIF: span = n/2 .. 1
  for (int ls = logn - 1; ls >= 0; --ls) {
    __syncthreads();
    const int span = 1 << ls;
    const int tstride = half >> ls;   // n / (2 span)
    for (int b = threadIdx.x; b < half; b += blockDim.x) {
      const int j = b & (span - 1);
      const int i0 = ((b >> ls) << (ls + 1)) + j;
      const int i1 = i0 + span;
      const double2 u = z[i0], v = z[i1];
      z[i0] = make_double2(u.x + v.x, u.y + v.y);
      z[i1] = cmul(make_double2(u.x - v.x, u.y - v.y), tw[j * tstride]);
    }
  }
  __syncthreads();
  // symbol (2 i k / n) with the 1/n of the inverse folded in; k = bitrev(pos)
  const double scale = 2.0 / ((double)n * (double)n);
  for (int pos = threadIdx.x; pos < n; pos += blockDim.x) {
    const int k = (int)(__brev((unsigned)pos) >> (32 - logn));
    const int ks = (k < half) ? k : ((k == half) ? 0 : k - n);
    const double c = scale * (double)ks;
    const double2 v = z[pos];
    z[pos] = make_double2(-c * v.y, c * v.x);
  }
  // inverse DIT: span = 1 .. n/2, conjugate twiddles
  for (int ls = 0; ls < logn; ++ls) {
    __syncthreads();
    const int span = 1 << ls;
    const int tstride = half >> ls;
    for (int b = threadIdx.x; b < half; b += blockDim.x) {
      const int j = b & (span - 1);
      const int i0 = ((b >> ls) << (ls + 1)) + j;
      const int i1 = i0 + span;
      const double2 u = z[i0];
      const double2 v = cmulc(z[i1], tw[j * tstride]);
      z[i0] = make_double2(u.x + v.x, u.y + v.y);
      z[i1] = make_double2(u.x - v.x, u.y - v.y);
    }
  }
  __syncthreads();
  double* ya = y + oa;
  double* yb = y + ob;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const double2 v = z[p];
    ya[p] += sign * v.x;
    if (hasb) yb[p] += sign * v.y;
  }
}

// direct fallback: y_p += sign * sum_q b_{(p-q) mod n} x_q
__global__ __launch_bounds__(256) void k_circulant_direct(const double* __restrict__ x, double* __restrict__ y,
                                                          const int64_t* __restrict__ offs, int n, double sign,
                                                          const double* __restrict__ b) {
  const int v = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double* xv = x + offs[v];
  double acc = 0.0;
  for (int q = 0; q < n; ++q) {
    int d = p - q;
    d += (d < 0) ? n : 0;
    acc = __builtin_fma(b[d], xv[q], acc);
  }
  y[offs[v] + p] += sign * acc;
}

int ilog2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

}  // namespace

bool circulant_uses_fft(int64_t n) { return n >= 2 && n <= kFftMaxN && (n & (n - 1)) == 0; }

// tw must hold n/2 double2 (FFT) or n doubles (direct fallback)
hipError_t launch_twiddles(double2* tw, int64_t n, hipStream_t st) {
  if (circulant_uses_fft(n)) {
    const int64_t h = n / 2;
    k_twiddles<<<(unsigned)((h + 255) / 256), 256, 0, st>>>(tw, (int)n);
  } else {
    k_circ_column<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(reinterpret_cast<double*>(tw), (int)n);
  }
  return hipGetLastError();
}

hipError_t launch_circulant(const double* x, double* y, const int64_t* offs, int nvec, int64_t n, double sign,
                            const double2* twiddle, hipStream_t st) {
  if (nvec <= 0) return hipSuccess;
  if (circulant_uses_fft(n)) {
    const unsigned pairs = (unsigned)((nvec + 1) / 2);
    const size_t lds = (size_t)n * sizeof(double2);
    k_circulant_fft<<<pairs, kFftThreads, lds, st>>>(x, y, offs, (int)n, ilog2(n), nvec, sign, twiddle);
  } else {
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)nvec);
    k_circulant_direct<<<grid, 256, 0, st>>>(x, y, offs, (int)n, sign, reinterpret_cast<const double*>(twiddle));
  }
  return hipGetLastError();
}

}  // namespace gnk

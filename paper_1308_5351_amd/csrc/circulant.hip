// Circulant blocks of the discretised singular operator M (paper Sec. 3.3):
//   (Lhat x) restricted to component k = L x_k,
//   L_pq = (-1)^(p-q) (1/n) cot((p-q) pi / n) (p != q), L_pp = 0.
// L is circulant, so L x_k = ifft(fft(b) .* fft(x_k)) (eq. (e:L-bs)) with b its
// first column; fft(b)_k equals 2 i k / n for the signed frequency |k| < n/2
// and 0 at k = n/2, so the symbol is applied in closed form.
//
// gfx950 mapping: each complex vector carries a PAIR of real length-n columns
// (two components, or two right-hand sides): because L is a real matrix,
// L (x_a + i x_b) = L x_a + i L x_b, so one complex FFT carries two real
// columns with no post-processing. A workgroup holds up to 2048 complex
// elements (whole vectors; fewer when that leaves the chip short of
// workgroups) in LDS: a decimation-in-frequency
// transform (natural order in, bit-reversed out), the symbol multiply in
// bit-reversed order, then a decimation-in-time inverse (bit-reversed in,
// natural out), so no permutation pass is needed. The radix-2 stages run
// three at a time on eight register-resident elements per thread, so a
// length-2048 product takes 7 trips through LDS instead of 24; the first pass
// reads x and the last adds into y directly.
// Global traffic is one read of x and one read-modify-write of y per element.
// The vectors are given as a list of flat offsets, so one launch covers every
// component of every column (and of every domain with this n).
// Powers of two up to 4096 use the FFT; other even n use a direct O(n^2)
// circulant product with the closed-form first column.
#include <algorithm>
#include <vector>

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

// Radix-2 stages fused F at a time: a group of 2^F elements at stride q,
// i0 + m q (m < 2^F), held in registers while the F stages act on it. DIF
// stages run with spans q 2^(F-1) .. q, DIT stages with spans q .. q 2^(F-1);
// each butterfly is the radix-2 one of its stage (twiddle index (i mod span)
// * n / (2 span)), so the transform and its bit-reversed middle order are
// those of the plain radix-2 passes. In a stage whose partners are h apart,
// the twiddles of the group are w_r = tw[j ts] exp(-i pi r / h), r < h <= 4:
// one table load per stage, the rest constant rotations.
template <int R, int H>
__device__ __forceinline__ double2 rotate(double2 b) {
  static_assert(R < H && H <= 4, "rotations for radix up to 8");
  if constexpr (R == 0) {
    return b;
  } else if constexpr (2 * R == H) {
    return make_double2(b.y, -b.x);                        // * (-i)
  } else {
    constexpr double c = 0.70710678118654752440;           // cos(pi/4)
    constexpr double sr = (R == 1) ? c : -c;               // real part of exp(-i pi R/4)
    return make_double2(sr * b.x + c * b.y, sr * b.y - c * b.x);   // * (sr - i c)
  }
}

template <int F, int f, bool DIF, int M = 0>
__device__ __forceinline__ void stage(double2 (&v)[1 << F], double2 base) {
  if constexpr (M < (1 << F)) {
    constexpr int h = DIF ? (1 << (F - 1 - f)) : (1 << f);
    if constexpr ((M & h) == 0) {
      const double2 w = rotate<(M & (h - 1)), h>(base);
      const double2 u = v[M];
      if constexpr (DIF) {
        const double2 t = v[M + h];
        v[M] = make_double2(u.x + t.x, u.y + t.y);
        v[M + h] = cmul(make_double2(u.x - t.x, u.y - t.y), w);
      } else {
        const double2 t = cmulc(v[M + h], w);
        v[M] = make_double2(u.x + t.x, u.y + t.y);
        v[M + h] = make_double2(u.x - t.x, u.y - t.y);
      }
    }
    stage<F, f, DIF, M + 1>(v, base);
  }
}

template <int F, bool DIF, int f = 0>
__device__ __forceinline__ void group_stages(double2 (&v)[1 << F], int j, int q, int half,
                                             const double2* __restrict__ tw) {
  if constexpr (f < F) {
    constexpr int h = DIF ? (1 << (F - 1 - f)) : (1 << f);
    const double2 base = tw[j * (half / (q * h))];
    stage<F, f, DIF>(v, base);
    group_stages<F, DIF, f + 1>(v, j, q, half, tw);
  }
}

// Complex elements per workgroup: P = kFftElems / n vectors of length n (one
// for n >= kFftElems), each carrying two real columns.
constexpr int kFftElems = 2048;

struct FftArgs {
  const double* x;
  double* y;
  const int64_t* offs;
  int n, logn, V, P;
  double sign;
  const double2* tw;
};

// Every block length of one product in one launch: workgroups first[c] ..
// first[c + 1] - 1 take class c (the classes' vector lists, lengths, twiddles).
constexpr int kMaxCirc = 12;   // powers of two 2 .. 4096
struct FftMulti {
  FftArgs a[kMaxCirc];
  int first[kMaxCirc + 1];
  int nc;
};

// One pass of F fused stages over every group of the workgroup's P vectors.
// FIRST: the elements come from x (global), not LDS. SYMBOL: after the last
// DIF stage, multiply by the symbol (2 i k / n, with the 1/n of the inverse),
// k the bit reversal of the position. LAST: the results go to y (global,
// y += sign * result) instead of LDS. KEEPY (with FIRST, F = 3): also fetch
// the y values of the group into yk; HAVEY (with LAST, F = 3): add to those
// instead of fetching them. For n <= 2048 the first and the last pass both
// give each thread one group of eight elements at stride n/8, the same ones.
template <int F, bool DIF, bool FIRST, bool SYMBOL, bool LAST, bool KEEPY = false, bool HAVEY = false>
__device__ __forceinline__ void fft_pass(const FftArgs& A, double2* z, int q, int wg, double2 (&yk)[8]) {
  static_assert(!(KEEPY || HAVEY) || F == 3, "y is kept for passes of eight elements");
  const int n = A.n, half = n >> 1;
  const int per = n >> F;   // groups per vector
  for (int g = threadIdx.x; g < A.P * per; g += blockDim.x) {
    const int vl = g / per, gg = g - vl * per;
    const int blk = gg / q, j = gg - blk * q;
    const int i0 = (blk << F) * q + j;
    double2* zv = z + (size_t)vl * n;
    const int va = 2 * (wg * A.P + vl);
    double2 v[1 << F];
    // LAST: the y values to add to are fetched before the LDS reads and the
    // butterflies, so their latency overlaps that work
    double2 yv[LAST ? (1 << F) : 1];
    if constexpr (LAST && HAVEY) {
#pragma unroll
      for (int m = 0; m < (1 << F); ++m) yv[m] = yk[m];
    } else if constexpr (LAST) {
      const bool hasa = va < A.V, hasb = va + 1 < A.V;
      const double* ya = A.y + (hasa ? A.offs[va] : 0);
      const double* yb = A.y + (hasb ? A.offs[va + 1] : 0);
#pragma unroll
      for (int m = 0; m < (1 << F); ++m) {
        const int p = i0 + m * q;
        yv[m] = make_double2(hasa ? __builtin_nontemporal_load(ya + p) : 0.0, hasb ? __builtin_nontemporal_load(yb + p) : 0.0);
      }
    }
    if constexpr (FIRST) {
      const bool hasa = va < A.V, hasb = va + 1 < A.V;
      const double* xa = A.x + (hasa ? A.offs[va] : 0);
      const double* xb = A.x + (hasb ? A.offs[va + 1] : 0);
#pragma unroll
      for (int m = 0; m < (1 << F); ++m) {
        const int p = i0 + m * q;
        v[m] = make_double2(hasa ? __builtin_nontemporal_load(xa + p) : 0.0, hasb ? __builtin_nontemporal_load(xb + p) : 0.0);
      }
      if constexpr (KEEPY) {
        const double* ya = A.y + (hasa ? A.offs[va] : 0);
        const double* yb = A.y + (hasb ? A.offs[va + 1] : 0);
#pragma unroll
        for (int m = 0; m < (1 << F); ++m) {
          const int p = i0 + m * q;
          yk[m] = make_double2(hasa ? __builtin_nontemporal_load(ya + p) : 0.0, hasb ? __builtin_nontemporal_load(yb + p) : 0.0);
        }
      }
    } else {
#pragma unroll
      for (int m = 0; m < (1 << F); ++m) v[m] = zv[i0 + m * q];
    }
    group_stages<F, DIF>(v, j, q, half, A.tw);
    if constexpr (SYMBOL) {
      const double scale = 2.0 / ((double)n * (double)n);
#pragma unroll
      for (int m = 0; m < (1 << F); ++m) {
        const int pos = i0 + m * q;
        const int k = (int)(__brev((unsigned)pos) >> (32 - A.logn));
        const int ks = (k < half) ? k : ((k == half) ? 0 : k - n);
        const double c = scale * (double)ks;
        v[m] = make_double2(-c * v[m].y, c * v[m].x);
      }
    }
    if constexpr (LAST) {
      const bool hasa = va < A.V, hasb = va + 1 < A.V;
      double* ya = A.y + (hasa ? A.offs[va] : 0);
      double* yb = A.y + (hasb ? A.offs[va + 1] : 0);
#pragma unroll
      for (int m = 0; m < (1 << F); ++m) {
        const int p = i0 + m * q;
        if (hasa) __builtin_nontemporal_store(__builtin_fma(A.sign, v[m].x, yv[m].x), ya + p);
        if (hasb) __builtin_nontemporal_store(__builtin_fma(A.sign, v[m].y, yv[m].y), yb + p);
      }
    } else {
#pragma unroll
      for (int m = 0; m < (1 << F); ++m) zv[i0 + m * q] = v[m];
    }
  }
}

template <bool DIF, bool FIRST, bool SYMBOL, bool LAST>
__device__ __forceinline__ void fft_pass_f(int F, const FftArgs& A, double2* z, int q, int wg, double2 (&yk)[8]) {
  if (F == 3) fft_pass<3, DIF, FIRST, SYMBOL, LAST>(A, z, q, wg, yk);
  else if (F == 2) fft_pass<2, DIF, FIRST, SYMBOL, LAST>(A, z, q, wg, yk);
  else fft_pass<1, DIF, FIRST, SYMBOL, LAST>(A, z, q, wg, yk);
}

// y_k += sign * L x_k for the vectors listed in offs (V of them, length n, a
// power of two) of every class: workgroup b of a class takes its complex
// vectors b P .. b P + P - 1, vector c carrying the real columns 2c and 2c + 1.
// Forward DIF (natural -> bit-reversed) in passes of up to three fused stages,
// the first reading x, the last applying the symbol; inverse DIT
// (bit-reversed -> natural), the last pass adding into y. Between passes the
// vectors sit in LDS.
__global__ __launch_bounds__(kFftThreads) void k_circulant_fft(FftMulti M) {
  extern __shared__ double2 z[];
  int c = 0;
  while (c + 1 < M.nc && (int)blockIdx.x >= M.first[c + 1]) ++c;
  const FftArgs A = M.a[c];
  const int wg = (int)blockIdx.x - M.first[c];
  const int L = A.logn;
  const int np = (L + 2) / 3;   // passes per direction; all of 3 stages but the last (L - 3 (np - 1))
  // y fetched with x in the first pass (one group of eight per thread, n <= 2048,
  // at least two passes), so both reads are in flight together
  const bool early = np >= 2 && A.P * (A.n >> 3) <= (int)blockDim.x;
  double2 yk[8];
  // forward: pass t covers stages with spans n/2 >> 3t .. ; its smallest span is q
  int top = L;                  // stages above this pass
  for (int t = 0; t < np; ++t) {
    const int F = (t + 1 < np) ? 3 : L - 3 * (np - 1);
    const int q = 1 << (top - F);
    if (t > 0) __syncthreads();
    const bool first = t == 0, last = t + 1 == np;
    if (first && early) fft_pass<3, true, true, false, false, true>(A, z, q, wg, yk);
    else if (first && last) fft_pass_f<true, true, true, false>(F, A, z, q, wg, yk);
    else if (first) fft_pass_f<true, true, false, false>(F, A, z, q, wg, yk);
    else if (last) fft_pass_f<true, false, true, false>(F, A, z, q, wg, yk);
    else fft_pass_f<true, false, false, false>(F, A, z, q, wg, yk);
    top -= F;
  }
  // inverse: the short pass first (smallest spans), then passes of three
  int bottom = 0;
  for (int t = 0; t < np; ++t) {
    const int F = (t == 0) ? L - 3 * (np - 1) : 3;
    const int q = 1 << bottom;
    __syncthreads();
    if (t + 1 == np && early) fft_pass<3, false, false, false, true, false, true>(A, z, q, wg, yk);
    else if (t + 1 == np) fft_pass_f<false, false, false, true>(F, A, z, q, wg, yk);
    else fft_pass_f<false, false, false, false>(F, A, z, q, wg, yk);
    bottom += F;
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

hipError_t launch_circulant(const double* x, double* y, const CircClass* cls, int ncls, double sign, hipStream_t st) {
  // power-of-two lengths: one launch for all of them (chunks of kMaxCirc
  // classes), 2048 complex elements (P = 2048 / n whole vectors, one for
  // n >= 2048) per workgroup of 256 threads; other lengths: the direct product
  FftMulti M{};
  size_t lds = 0;
  int wgs = 0;
  auto flush = [&]() -> hipError_t {
    if (M.nc == 0) return hipSuccess;
    M.first[M.nc] = wgs;
    k_circulant_fft<<<(unsigned)wgs, kFftThreads, lds, st>>>(M);
    M = FftMulti{};
    lds = 0;
    wgs = 0;
    return hipGetLastError();
  };
  // longest vectors first: their workgroups take longest, so the short ones
  // fill the tail of the launch
  std::vector<int> order(ncls);
  for (int k = 0; k < ncls; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cls[a].n > cls[b].n; });
  for (int k : order) {
    const CircClass& C = cls[k];
    if (C.nvec <= 0) continue;
    if (circulant_uses_fft(C.n)) {
      const int64_t cvec = (C.nvec + 1) / 2;
      const int P = (int)std::max<int64_t>(1, kFftElems / C.n);
      M.a[M.nc] = FftArgs{x, y, C.offs, (int)C.n, ilog2(C.n), C.nvec, P, sign, C.tw};
      M.first[M.nc] = wgs;
      wgs += (int)((cvec + P - 1) / P);
      lds = std::max(lds, (size_t)P * C.n * sizeof(double2));
      if (++M.nc == kMaxCirc) {
        const hipError_t e = flush();
        if (e != hipSuccess) return e;
      }
    } else {
      dim3 grid((unsigned)((C.n + 255) / 256), (unsigned)C.nvec);
      k_circulant_direct<<<grid, 256, 0, st>>>(x, y, C.offs, (int)C.n, sign,
                                               reinterpret_cast<const double*>(C.tw));
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return flush();
}

}  // namespace gnk

// Host driver of libgnk: context and workspace, input validation, operator
// application, the device-resident restarted GMRES, and the C ABI entry points
// declared in include/gnk.h.
//
// Method (paper Sec. 3 and 4):
//   FBIE   : y = (D - diag(D1) + Lhat) gamma; solve (2I + diag(B1) - B) mu = -y;
//            h = [(D - diag(D1) + Lhat) mu - (2I + diag(B1) - B) gamma] / 2.
//   FBIEad : e from eq. (e:bve); solve (diag(e) + B^T + Phat) mu = gamma.
// Every product with B, D, B^T, D^T is one Cauchy sum S = E w followed by a
// per-node epilogue; the circulant blocks use the LDS FFT kernel.
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "gnk_internal.h"
#include "vec_kernels.inl"

struct gnk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int num_cu = 256;
  size_t ws_limit = 0;   // bytes, 0 = unlimited
  size_t ws_bytes = 0;
  bool log = false;
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  int64_t tw_n = -1;     // n of the cached circulant table
  // pipelined convergence read-back of the GMRES iterations
  int* pinned = nullptr;                 // host-pinned, one int per Arnoldi step
  double* pinned_rel = nullptr;          // host-pinned residual estimates (mixed switch)
  size_t pinned_rel_n = 0;
  std::vector<hipEvent_t> step_ev;       // one event per Arnoldi step
  // optional timing of the Cauchy-sum launches (HIP events on the context stream)
  bool prof = false;
  struct ProfRec {
    hipEvent_t a, b;
    int64_t N;
    int ncols;
    bool mixed;
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  gnk_prof prof_acc{};
};

namespace gnk {
namespace {

struct Fail {
  gnk_status st;
};

void set_err(gnk_ctx* c, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void set_err(gnk_ctx* c, const char* fmt, ...) {
  char b[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(b, sizeof b, fmt, ap);
  va_end(ap);
  c->err = b;
}

#define HIPCHK(ctx, x)                                                                       \
  do {                                                                                       \
    hipError_t e_ = (x);                                                                     \
    if (e_ != hipSuccess) {                                                                  \
      set_err(ctx, "%s failed: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, __LINE__);  \
      throw Fail{GNK_ERR_HIP};                                                               \
    }                                                                                        \
  } while (0)

#define LAUNCHCHK(ctx) HIPCHK(ctx, hipGetLastError())

template <class T>
T* ws(gnk_ctx* c, const std::string& name, size_t count) {
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  auto& b = c->bufs[name];
  if (b.bytes >= bytes) return static_cast<T*>(b.p);
  if (b.p) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipFree(b.p));
    c->ws_bytes -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  if (c->ws_limit && c->ws_bytes + bytes > c->ws_limit) {
    set_err(c, "workspace '%s' of %zu bytes exceeds the limit of %zu bytes", name.c_str(), bytes, c->ws_limit);
    throw Fail{GNK_ERR_OOM};
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_err(c, "hipMalloc of %zu bytes for '%s' failed", bytes, name.c_str());
    throw Fail{GNK_ERR_OOM};
  }
  b.p = p;
  b.bytes = bytes;
  c->ws_bytes += bytes;
  return static_cast<T*>(p);
}

unsigned nblocks(int64_t n, int t = kT) { return (unsigned)((n + t - 1) / t); }

// ----------------------------------------------------------- prepared domain
struct Prep {
  int64_t N = 0, n = 0, m1 = 0;
  const double2* eta = nullptr;
  const double2* etap = nullptr;
  const double2* etapp = nullptr;
  const double2* A = nullptr;
  const double2* Ap = nullptr;
  int c = 1;
  double2* rho = nullptr;   // eta'/A
  double* dB = nullptr;     // diag(B1)
  double* dD = nullptr;     // diag(D1)
  double* e = nullptr;      // vector e (adjoint equation)
  double2* tw = nullptr;    // circulant table
  CauchyPlan plan;
  // mixed precision (FP32 far tiles)
  CauchyPlan mplan;
  double4* sb = nullptr;    // 64-node source tile bounds
  double4* tb = nullptr;    // target tile bounds (64 * mplan.tpt nodes)
  double far2 = 4.0;
};

void check_domain(gnk_ctx* c, const gnk_domain* d, bool adjoint) {
  if (!d) {
    set_err(c, "domain is NULL");
    throw Fail{GNK_ERR_ARG};
  }
  if (d->m1 < 1 || d->n < 2) {
    set_err(c, "need m1 >= 1 and n >= 2 (got m1=%lld n=%lld)", (long long)d->m1, (long long)d->n);
    throw Fail{GNK_ERR_ARG};
  }
  if (d->n % 2) {
    set_err(c, "n must be even (got %lld)", (long long)d->n);
    throw Fail{GNK_ERR_ODD_N};
  }
  if (d->m1 * d->n > (int64_t)1 << 30) {
    set_err(c, "N = (m+1) n = %lld exceeds 2^30", (long long)(d->m1 * d->n));
    throw Fail{GNK_ERR_ARG};
  }
  if (!d->eta || !d->etap || !d->A) {
    set_err(c, "eta, etap and A are required");
    throw Fail{GNK_ERR_ARG};
  }
  if (adjoint && (!d->etapp || !d->Ap || (d->c != 1 && d->c != -1))) {
    set_err(c, "the adjoint equation needs etapp, Ap and c = +1 or -1");
    throw Fail{GNK_ERR_ARG};
  }
}

void validate_inputs(gnk_ctx* c, const Prep& P, bool adjoint, const double* x, int nrhs) {
  int* flags = ws<int>(c, "flags", 1);
  HIPCHK(c, hipMemsetAsync(flags, 0, sizeof(int), c->stream));
  k_validate<<<nblocks(P.N), kT, 0, c->stream>>>(P.eta, P.etap, P.A, adjoint ? P.etapp : nullptr,
                                                  adjoint ? P.Ap : nullptr, (int)P.N, adjoint ? 1 : 0, flags);
  LAUNCHCHK(c);
  if (x) {
    const int64_t len = P.N * nrhs;
    k_check_finite<<<nblocks(len), kT, 0, c->stream>>>(x, len, flags);
    LAUNCHCHK(c);
  }
  int h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (h & 1) {
    set_err(c, "non-finite value in the inputs");
    throw Fail{GNK_ERR_NONFINITE};
  }
  if (h & 2) {
    set_err(c, "A vanishes at a node");
    throw Fail{GNK_ERR_ZERO_A};
  }
  if (h & 4) {
    set_err(c, "eta' vanishes at a node (the adjoint equation divides by eta')");
    throw Fail{GNK_ERR_ZERO_ETAP};
  }
}

Prep make_prep(gnk_ctx* c, const gnk_domain* d, bool adjoint) {
  Prep P;
  P.m1 = d->m1;
  P.n = d->n;
  P.N = d->m1 * d->n;
  P.eta = static_cast<const double2*>(d->eta);
  P.etap = static_cast<const double2*>(d->etap);
  P.etapp = static_cast<const double2*>(d->etapp);
  P.A = static_cast<const double2*>(d->A);
  P.Ap = static_cast<const double2*>(d->Ap);
  P.c = d->c;
  P.plan = plan_cauchy(P.N, 1, c->num_cu);
  (void)adjoint;
  return P;
}

double2* cauchy_parts(gnk_ctx* c, const Prep& P, int ncols) {
  return ws<double2>(c, "parts", (size_t)P.plan.splits * ncols * P.N);
}

hipEvent_t pool_event(gnk_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(c, hipEventCreate(&e));
  return e;
}

// One Cauchy-sum launch (all column groups), timed when profiling is on.
void cauchy(gnk_ctx* c, const double2* rec, int64_t N, int ncols, const CauchyPlan& plan, double2* parts) {
  if (!c->prof) {
    HIPCHK(c, launch_cauchy_fp64(rec, N, ncols, plan, parts, c->stream));
    return;
  }
  gnk_ctx::ProfRec r{pool_event(c), pool_event(c), N, ncols, false};
  HIPCHK(c, hipEventRecord(r.a, c->stream));
  HIPCHK(c, launch_cauchy_fp64(rec, N, ncols, plan, parts, c->stream));
  HIPCHK(c, hipEventRecord(r.b, c->stream));
  c->prof_pending.push_back(r);
}

void cauchy_mixed(gnk_ctx* c, const MixedArgs& m, int64_t N, int ncols, const CauchyPlan& plan, double2* parts) {
  if (!c->prof) {
    HIPCHK(c, launch_cauchy_mixed(m, N, ncols, plan, parts, c->stream));
    return;
  }
  gnk_ctx::ProfRec r{pool_event(c), pool_event(c), N, ncols, true};
  HIPCHK(c, hipEventRecord(r.a, c->stream));
  HIPCHK(c, launch_cauchy_mixed(m, N, ncols, plan, parts, c->stream));
  HIPCHK(c, hipEventRecord(r.b, c->stream));
  c->prof_pending.push_back(r);
}

void ensure_twiddles(gnk_ctx* c, Prep& P) {
  const size_t cnt = circulant_uses_fft(P.n) ? (size_t)P.n / 2 : (size_t)(P.n + 1) / 2;
  P.tw = ws<double2>(c, "twiddle", cnt + 1);
  if (c->tw_n != P.n) {
    HIPCHK(c, launch_twiddles(P.tw, P.n, c->stream));
    c->tw_n = P.n;
  }
}

// S = E w for one complex column w (setup products)
double2* cauchy_single(gnk_ctx* c, const Prep& P, const double2* w) {
  double2* rec = ws<double2>(c, "rec", (size_t)P.N * 2);
  k_pack_records<<<nblocks(P.N), kT, 0, c->stream>>>(P.eta, w, (int)P.N, 1, rec);
  LAUNCHCHK(c);
  double2* parts = cauchy_parts(c, P, 1);
  cauchy(c, rec, P.N, 1, P.plan, parts);
  return parts;
}

// rho = eta'/A and, from S = E(rho), diag(B1) and diag(D1)
void setup_fbie(gnk_ctx* c, Prep& P) {
  P.rho = ws<double2>(c, "rho", P.N);
  P.dB = ws<double>(c, "dB", P.N);
  P.dD = ws<double>(c, "dD", P.N);
  k_rho<<<nblocks(P.N), kT, 0, c->stream>>>(P.etap, P.A, P.rho, (int)P.N);
  LAUNCHCHK(c);
  double2* parts = cauchy_single(c, P, P.rho);
  k_diag_fbie<<<nblocks(P.N), kT, 0, c->stream>>>(parts, P.plan.splits, 1, P.A, (int)P.N, 2.0 / P.n, P.dB,
                                                   P.dD);
  LAUNCHCHK(c);
}

// e of eq. (e:bve) from S = E eta'
void setup_fbiead(gnk_ctx* c, Prep& P) {
  if (!P.rho) {
    P.rho = ws<double2>(c, "rho", P.N);
    k_rho<<<nblocks(P.N), kT, 0, c->stream>>>(P.etap, P.A, P.rho, (int)P.N);
    LAUNCHCHK(c);
  }
  P.e = ws<double>(c, "evec", P.N);
  double2* parts = cauchy_single(c, P, P.etap);
  k_evec<<<nblocks(P.N), kT, 0, c->stream>>>(parts, P.plan.splits, P.etap, P.etapp, P.A, P.Ap, (int)P.N,
                                              2.0 / P.n, (double)P.c, P.e);
  LAUNCHCHK(c);
}

// tile bounds for the mixed-precision pair kernel
void setup_mixed(gnk_ctx* c, Prep& P) {
  P.mplan = plan_cauchy(P.N, 1, c->num_cu, 256);
  const int ttile = 64 * P.mplan.tpt;
  P.sb = ws<double4>(c, "sbnd", (size_t)(P.N + 63) / 64);
  P.tb = ws<double4>(c, "tbnd", (size_t)(P.N + ttile - 1) / ttile);
  HIPCHK(c, launch_tile_bounds(P.eta, P.N, 0, 64, P.sb, c->stream));
  HIPCHK(c, launch_tile_bounds(P.eta, P.N, 0, ttile, P.tb, c->stream));
  double theta = 1.0;
  if (const char* e = getenv("GNK_MIXED_THETA")) theta = atof(e);
  P.far2 = (1.0 + theta) * (1.0 + theta);
}

// --------------------------------------------------------- operator product
// y = op(x) for nrhs columns. scale/xout: optional per-column scaling of x
// written back (GMRES normalisation); active: optional per-column GMRES mask.
struct ApplyArgs {
  const double* scale = nullptr;
  double* xout = nullptr;
  const int* active = nullptr;
  bool mixed = false;      // FP32 far tiles (needs setup_mixed)
};

void apply_op(gnk_ctx* c, Prep& P, int op, const double* x, int nrhs, double* y, const ApplyArgs& a = {}) {
  const double two_n = 2.0 / (double)P.n;
  const bool need_mean = (op == GNK_OP_GB || op == GNK_OP_GB_T);
  if (op == GNK_OP_LHAT) {
    ensure_twiddles(c, P);
    HIPCHK(c, hipMemsetAsync(y, 0, sizeof(double) * P.N * nrhs, c->stream));
    HIPCHK(c, launch_circulant(x, y, P.m1, P.n, nrhs, 1.0, P.tw, c->stream));
    return;
  }
  // weight factor C: rho for B x, D x, B^T... (see eqs. (e:(I-B)x), (e:hD-bt), (e:BTx))
  const double2* Cw = nullptr;
  const double2* Cout = nullptr;
  double a0 = 0.0, dsign = 0.0, cI = 0.0, cR = 0.0;
  const double* dg = nullptr;
  switch (op) {
    case GNK_OP_FB:   // 2x + diag(B1) x - B x,  B x = -(2/n) Im(A E(rho x))
      Cw = P.rho; Cout = P.A; a0 = 2.0; dg = P.dB; dsign = 1.0; cI = two_n; break;
    case GNK_OP_FC:   // D x - diag(D1) x (+ Lhat x),  D x = -(2/n) Re(A E(rho x))
      Cw = P.rho; Cout = P.A; dg = P.dD; dsign = -1.0; cR = -two_n; break;
    case GNK_OP_GB:   // e x + B^T x + Phat x,  B^T x = (2/n) Im(rho E(A x))
      Cw = P.A; Cout = P.rho; dg = P.e; dsign = 1.0; cI = two_n; break;
    case GNK_OP_FB_T: // 2x + diag(B1) x - B^T x
      Cw = P.A; Cout = P.rho; a0 = 2.0; dg = P.dB; dsign = 1.0; cI = -two_n; break;
    case GNK_OP_FC_T: // D^T x - diag(D1) x - Lhat x,  D^T x = (2/n) Re(rho E(A x))
      Cw = P.A; Cout = P.rho; dg = P.dD; dsign = -1.0; cR = two_n; break;
    case GNK_OP_GB_T: // e x + B x + Phat x
      Cw = P.rho; Cout = P.A; dg = P.e; dsign = 1.0; cI = -two_n; break;
    default:
      set_err(c, "unknown operator %d", op);
      throw Fail{GNK_ERR_ARG};
  }
  double2* rec = ws<double2>(c, "rec", (size_t)P.N * (nrhs + 1));
  double* mean = need_mean ? ws<double>(c, "mean", (size_t)P.m1 * nrhs) : nullptr;
  dim3 gw((unsigned)P.m1, (unsigned)nrhs);
  k_weights<<<gw, kT, 0, c->stream>>>(P.eta, Cw, x, a.scale, a.active, a.xout, rec, (int)P.N, (int)P.n, (int)P.m1,
                                      nrhs + 1, 0, 0, mean);
  LAUNCHCHK(c);
  const double* xin = a.xout ? a.xout : x;
  double2* parts;
  int splits;
  if (a.mixed) {
    float2* rec32 = ws<float2>(c, "rec32", (size_t)P.N * (nrhs + 1));
    HIPCHK(c, launch_records32(rec, P.sb, P.N, nrhs, rec32, c->stream));
    parts = ws<double2>(c, "parts", (size_t)P.mplan.splits * nrhs * P.N);
    splits = P.mplan.splits;
    MixedArgs m{rec, rec32, P.sb, P.tb, P.far2};
    cauchy_mixed(c, m, P.N, nrhs, P.mplan, parts);
  } else {
    parts = cauchy_parts(c, P, nrhs);
    splits = P.plan.splits;
    cauchy(c, rec, P.N, nrhs, P.plan, parts);
  }
  dim3 ge(nblocks(P.N), (unsigned)nrhs);
  k_epilogue<<<ge, kT, 0, c->stream>>>(parts, splits, nrhs, 0, xin, Cout, dg, a0, dsign, cI, cR, mean,
                                       (int)P.n, (int)P.m1, a.active, y, (int)P.N);
  LAUNCHCHK(c);
  if (op == GNK_OP_FC || op == GNK_OP_FC_T) {
    ensure_twiddles(c, P);
    HIPCHK(c, launch_circulant(xin, y, P.m1, P.n, nrhs, op == GNK_OP_FC ? 1.0 : -1.0, P.tw, c->stream));
  }
}

// ------------------------------------------------------------------ GMRES
struct GmresOut {
  std::vector<gnk_info> info;
  bool all_converged = false;
};

// Restarted GMRES. With `mixed`, the Arnoldi products switch to the
// mixed-precision pair kernel once the residual estimate of every column is
// below o.inner_tol (relaxed products: an error of relative size e in a
// product made when the residual is r perturbs the final residual by about
// e*r, so FP32 far tiles are harmless once r <= tol / e). The residual that
// starts every cycle is always recomputed with the FP64 product, so each
// restart is a step of FP64 iterative refinement.
GmresOut gmres(gnk_ctx* c, Prep& P, int op, const double* b, int nrhs, const gnk_opts& o, double* x,
               bool mixed = false) {
  const ApplyArgs am;   // FP64 products for every true residual
  const int64_t N = P.N;
  const int restart = o.restart;
  const int ldp = kMaxRestart + 1;
  // vector-kernel blocking: 256..kMaxChunk elements per block, about 256 blocks
  const int per_blk = (int)std::max<int64_t>(kT, std::min<int64_t>(kMaxChunk, (N + 255) / 256));
  const int nblk = (int)((N + per_blk - 1) / per_blk);

  double* V = ws<double>(c, "V", (size_t)(restart + 1) * nrhs * N);
  double* P1 = ws<double>(c, "gmP1", (size_t)nrhs * nblk * ldp);
  double* P2 = ws<double>(c, "gmP2", (size_t)nrhs * nblk * ldp);
  GmresState st;
  st.ldh = restart + 1;
  st.hstride = st.ldh * restart;
  double* dbl = ws<double>(c, "gmdbl", (size_t)nrhs * (4 + st.hstride + 2 * kMaxRestart + (kMaxRestart + 1) +
                                                      kMaxRestart));
  int* ints = ws<int>(c, "gmint", (size_t)nrhs * 5 + 1);
  {
    double* q = dbl;
    st.bnorm = q; q += nrhs;
    st.true_relres = q; q += nrhs;
    st.relres = q; q += nrhs;
    st.invbeta = q; q += nrhs;
    st.H = q; q += (size_t)nrhs * st.hstride;
    st.cs = q; q += (size_t)nrhs * kMaxRestart;
    st.sn = q; q += (size_t)nrhs * kMaxRestart;
    st.g = q; q += (size_t)nrhs * (kMaxRestart + 1);
    st.y = q;
    int* r = ints;
    st.active = r; r += nrhs;
    st.converged = r; r += nrhs;
    st.kdim = r; r += nrhs;
    st.inner_it = r; r += nrhs;
    st.live = r;
  }
  const unsigned tb = (unsigned)std::min(1024, ((nrhs + 63) / 64) * 64);
  k_gmres_init<<<1, tb, 0, c->stream>>>(nrhs, st);
  LAUNCHCHK(c);
  dim3 gv((unsigned)nblk, (unsigned)nrhs);
  k_norm_partial<<<gv, kT, 0, c->stream>>>(b, (int)N, per_blk, P1, ldp);
  LAUNCHCHK(c);
  k_bnorm<<<1, tb, 0, c->stream>>>(P1, nblk, ldp, nrhs, st);
  LAUNCHCHK(c);

  // r0 = b - A x0 into V_0
  const size_t colbytes = sizeof(double) * N * nrhs;
  if (o.x0) {
    if (o.x0 != x) HIPCHK(c, hipMemcpyAsync(x, o.x0, colbytes, hipMemcpyDeviceToDevice, c->stream));
    apply_op(c, P, op, x, nrhs, V, am);
    k_residual<<<gv, kT, 0, c->stream>>>(b, V, (int)N, per_blk, P1, ldp);
  } else {
    HIPCHK(c, hipMemsetAsync(x, 0, colbytes, c->stream));
    HIPCHK(c, hipMemcpyAsync(V, b, colbytes, hipMemcpyDeviceToDevice, c->stream));
    k_norm_partial<<<gv, kT, 0, c->stream>>>(V, (int)N, per_blk, P1, ldp);
  }
  LAUNCHCHK(c);
  k_cycle_start<<<1, tb, 0, c->stream>>>(P1, nblk, ldp, nrhs, o.tol, st);
  LAUNCHCHK(c);

  std::vector<int> outer(nrhs, 0);
  std::vector<int> conv(nrhs, 0);
  std::vector<int> mixed_cycles(nrhs, 0);
  bool mixed_now = false;
  if (!c->pinned) HIPCHK(c, hipHostMalloc((void**)&c->pinned, sizeof(int) * (kMaxRestart + 1), 0));
  if (c->pinned_rel_n < (size_t)nrhs * kMaxRestart) {
    if (c->pinned_rel) HIPCHK(c, hipHostFree(c->pinned_rel));
    c->pinned_rel = nullptr;
    HIPCHK(c, hipHostMalloc((void**)&c->pinned_rel, sizeof(double) * nrhs * kMaxRestart, 0));
    c->pinned_rel_n = (size_t)nrhs * kMaxRestart;
  }
  while ((int)c->step_ev.size() < kMaxRestart) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->step_ev.push_back(e);
  }
  for (int cyc = 0; cyc < o.maxit; ++cyc) {
    int live = 0;
    HIPCHK(c, hipMemcpyAsync(&live, st.live, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(conv.data(), st.converged, sizeof(int) * nrhs, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (live == 0) break;
    for (int r = 0; r < nrhs; ++r)
      if (!conv[r]) {
        outer[r] += 1;
        if (mixed_now) mixed_cycles[r] += 1;
      }
    // Arnoldi steps. The host looks one step behind the device: before
    // enqueuing step l+1 it waits for step l-1 and reads how many columns are
    // still iterating, so the queue never drains and at most one speculative
    // step runs (fully masked) after the last column stops.
    for (int l = 0; l < restart; ++l) {
      double* vl = V + (size_t)l * nrhs * N;
      double* w = V + (size_t)(l + 1) * nrhs * N;
      ApplyArgs aa;
      aa.scale = st.invbeta;
      aa.xout = vl;
      aa.active = st.active;
      aa.mixed = mixed && mixed_now;
      apply_op(c, P, op, vl, nrhs, w, aa);
      k_gs_dot<<<gv, kT, 0, c->stream>>>(V, l + 1, w, (int)N, nrhs, per_blk, st.active, P1, ldp);
      LAUNCHCHK(c);
      k_gs_update<<<gv, kT, 0, c->stream>>>(V, l + 1, w, (int)N, nrhs, per_blk, st.active, P1, P2, ldp, st.H,
                                            st.ldh, st.hstride, l, 0, 1);
      LAUNCHCHK(c);
      k_gs_update<<<gv, kT, 0, c->stream>>>(V, l + 1, w, (int)N, nrhs, per_blk, st.active, P2, P1, ldp, st.H,
                                            st.ldh, st.hstride, l, 1, 0);
      LAUNCHCHK(c);
      k_arnoldi_finish<<<(unsigned)nrhs, 64, 0, c->stream>>>(P1, nblk, ldp, l, restart, o.tol, st);
      LAUNCHCHK(c);
      HIPCHK(c, hipMemcpyAsync(c->pinned + l, st.live, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      if (mixed && !mixed_now)
        HIPCHK(c, hipMemcpyAsync(c->pinned_rel + (size_t)l * nrhs, st.relres, sizeof(double) * nrhs,
                                 hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipEventRecord(c->step_ev[l], c->stream));
      if (l >= 1) {
        HIPCHK(c, hipEventSynchronize(c->step_ev[l - 1]));
        if (c->pinned[l - 1] == 0) break;
        if (mixed && !mixed_now) {
          double mx = 0.0;
          for (int r = 0; r < nrhs; ++r) mx = std::max(mx, c->pinned_rel[(size_t)(l - 1) * nrhs + r]);
          if (mx <= o.inner_tol) mixed_now = true;
        }
      }
    }
    k_backsolve<<<(unsigned)nrhs, 64, 0, c->stream>>>(st);
    LAUNCHCHK(c);
    k_xupdate<<<dim3(nblocks(N), (unsigned)nrhs), kT, 0, c->stream>>>(V, x, (int)N, nrhs, st);
    LAUNCHCHK(c);
    // true residual of the new iterate (FP64 product) and the next cycle's start
    apply_op(c, P, op, x, nrhs, V, am);
    k_residual<<<gv, kT, 0, c->stream>>>(b, V, (int)N, per_blk, P1, ldp);
    LAUNCHCHK(c);
    k_cycle_start<<<1, tb, 0, c->stream>>>(P1, nblk, ldp, nrhs, o.tol, st);
    LAUNCHCHK(c);
    if (c->log) {
      std::vector<double> tr(nrhs);
      HIPCHK(c, hipMemcpyAsync(tr.data(), st.true_relres, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      double mx = 0;
      for (double v : tr) mx = std::max(mx, v);
      fprintf(stderr, "[gnk] op %d cycle %d max true relres %.3e\n", op, cyc + 1, mx);
    }
  }
  GmresOut out;
  out.info.resize(nrhs);
  std::vector<double> rel(nrhs), trel(nrhs);
  std::vector<int> inner(nrhs);
  HIPCHK(c, hipMemcpyAsync(conv.data(), st.converged, sizeof(int) * nrhs, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(rel.data(), st.relres, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(trel.data(), st.true_relres, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(inner.data(), st.inner_it, sizeof(int) * nrhs, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out.all_converged = true;
  for (int r = 0; r < nrhs; ++r) {
    gnk_info& I = out.info[r];
    I.flag = conv[r] ? 0 : 1;
    I.outer_it = outer[r];
    I.inner_it = inner[r];
    I.refine_steps = mixed_cycles[r];
    I.relres = rel[r];
    I.true_relres = trel[r];
    if (!conv[r]) out.all_converged = false;
  }
  return out;
}

gnk_opts resolve_opts(gnk_ctx* c, const gnk_opts* o) {
  gnk_opts r{};
  r.restart = 25;
  r.maxit = 40;
  r.tol = 1e-12;
  r.prec = GNK_FP64;
  r.inner_tol = 0.0;
  r.max_refine = 0;
  r.x0 = nullptr;
  if (o) r = *o;
  // mixed products once the residual estimate is below tol / 1e-8 (their
  // relative error is below 1e-8), but not before 1e-4
  if (r.inner_tol <= 0) r.inner_tol = std::min(1e-4, r.tol * 1e8);
  if (r.restart < 1 || r.restart > kMaxRestart || r.maxit < 1 || !(r.tol > 0.0) || r.tol >= 1.0 ||
      (r.prec != GNK_FP64 && r.prec != GNK_MIXED)) {
    set_err(c, "bad options: restart %d (1..%d), maxit %d (>=1), tol %g (0..1), prec %d", r.restart, kMaxRestart,
            r.maxit, r.tol, r.prec);
    throw Fail{GNK_ERR_ARG};
  }
  return r;
}

template <class F>
gnk_status guarded(gnk_ctx* c, F&& f) {
  if (!c) return GNK_ERR_ARG;
  c->err.clear();
  try {
    HIPCHK(c, hipSetDevice(c->device));
    return f();
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    set_err(c, "host allocation failed");
    return GNK_ERR_OOM;
  }
}

}  // namespace
}  // namespace gnk

using namespace gnk;

extern "C" {

const char* gnk_version(void) { return "gnk 0.1.0 (gfx950, FP64 direct Cauchy sums)"; }

gnk_status gnk_create(gnk_ctx** out, int device) {
  if (!out) return GNK_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return GNK_ERR_HIP;
  }
  auto* c = new (std::nothrow) gnk_ctx();
  if (!c) return GNK_ERR_OOM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return GNK_ERR_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cu = prop.multiProcessorCount;
  if (const char* s = getenv("GNK_WORKSPACE_MB")) c->ws_limit = (size_t)atoll(s) << 20;
  if (const char* s = getenv("GNK_LOG")) c->log = atoi(s) != 0;
  *out = c;
  return GNK_OK;
}

gnk_status gnk_destroy(gnk_ctx* c) {
  if (!c) return GNK_ERR_ARG;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (auto& kv : c->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto e : c->step_ev) (void)hipEventDestroy(e);
  for (auto& r : c->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->pinned_rel) (void)hipHostFree(c->pinned_rel);
  delete c;
  return GNK_OK;
}

gnk_status gnk_set_stream(gnk_ctx* c, void* s) {
  if (!c) return GNK_ERR_ARG;
  c->stream = static_cast<hipStream_t>(s);
  return GNK_OK;
}

const char* gnk_last_error(const gnk_ctx* c) { return c ? c->err.c_str() : "null context"; }

gnk_status gnk_profile(gnk_ctx* c, int enable) {
  if (!c) return GNK_ERR_ARG;
  c->prof = enable != 0;
  return GNK_OK;
}

gnk_status gnk_profile_read(gnk_ctx* c, gnk_prof* out, int reset) {
  return guarded(c, [&]() -> gnk_status {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto& r : c->prof_pending) {
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, r.a, r.b));
      const double pairs = (double)r.N * (double)(r.N - 1);
      gnk_prof& A = c->prof_acc;
      A.launches += 1;
      A.ms += ms;
      A.pair_cols += pairs * r.ncols;
      A.flops += pairs * (16.0 + 8.0 * (r.ncols - 1));
      if (r.mixed) {
        A.launches_mixed += 1;
        A.ms_mixed += ms;
        A.pair_cols_mixed += pairs * r.ncols;
      } else if (r.ncols == 1) {
        A.launches1 += 1;
        A.ms1 += ms;
        A.pairs1 += pairs;
      }
      c->ev_pool.push_back(r.a);
      c->ev_pool.push_back(r.b);
    }
    c->prof_pending.clear();
    if (out) *out = c->prof_acc;
    if (reset) c->prof_acc = gnk_prof{};
    return GNK_OK;
  });
}

gnk_status gnk_cauchy_sum(gnk_ctx* c, int64_t N, const void* eta, const void* w, int nrhs, void* S) {
  return guarded(c, [&]() -> gnk_status {
    if (N < 1 || N > ((int64_t)1 << 30) || nrhs < 1 || !eta || !w || !S || w == S) {
      set_err(c, "bad arguments to gnk_cauchy_sum");
      throw Fail{GNK_ERR_ARG};
    }
    CauchyPlan plan = plan_cauchy(N, nrhs, c->num_cu);
    double2* parts = ws<double2>(c, "parts", (size_t)plan.splits * nrhs * N);
    double2* rec = ws<double2>(c, "rec", (size_t)N * (nrhs + 1));
    k_pack_records<<<nblocks(N), kT, 0, c->stream>>>(static_cast<const double2*>(eta),
                                                      static_cast<const double2*>(w), (int)N, nrhs, rec);
    LAUNCHCHK(c);
    cauchy(c, rec, N, nrhs, plan, parts);
    // reduce the splits in order: S[r*N + i] = sum_g parts
    // (reuse the epilogue-free path: a dedicated small kernel)
    k_reduce_parts<<<dim3(nblocks(N), (unsigned)nrhs), kT, 0, c->stream>>>(parts, plan.splits, nrhs, (int)N,
                                                                           static_cast<double2*>(S));
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GNK_OK;
  });
}

gnk_status gnk_apply(gnk_ctx* c, const gnk_domain* d, int op, int prec, const double* x, int nrhs, double* y) {
  return guarded(c, [&]() -> gnk_status {
    const bool adj = (op == GNK_OP_GB || op == GNK_OP_GB_T);
    check_domain(c, d, adj);
    if (!x || !y || x == y || nrhs < 1 || op < 0 || op > GNK_OP_LHAT || (prec != GNK_FP64 && prec != GNK_MIXED)) {
      set_err(c, "bad arguments to gnk_apply");
      throw Fail{GNK_ERR_ARG};
    }
    Prep P = make_prep(c, d, adj);
    validate_inputs(c, P, adj, x, nrhs);
    if (op != GNK_OP_LHAT) {
      setup_fbie(c, P);
      if (adj) setup_fbiead(c, P);
    }
    ApplyArgs a;
    if (prec == GNK_MIXED && op != GNK_OP_LHAT) {
      setup_mixed(c, P);
      a.mixed = true;
    }
    apply_op(c, P, op, x, nrhs, y, a);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GNK_OK;
  });
}

gnk_status gnk_fbie(gnk_ctx* c, const gnk_domain* d, const double* gam, int nrhs, const gnk_opts* opts, double* mu,
                    double* h, gnk_info* info) {
  return guarded(c, [&]() -> gnk_status {
    check_domain(c, d, false);
    if (!gam || !mu || nrhs < 1 || nrhs > 1024 || mu == gam || h == gam || (h && h == mu)) {
      set_err(c, "bad arguments to gnk_fbie");
      throw Fail{GNK_ERR_ARG};
    }
    gnk_opts o = resolve_opts(c, opts);
    Prep P = make_prep(c, d, false);
    validate_inputs(c, P, false, gam, nrhs);
    const int64_t N = P.N;
    const double two_n = 2.0 / (double)P.n;
    // rho = eta'/A; one Cauchy launch for E(rho) and E(rho gamma)
    P.rho = ws<double2>(c, "rho", N);
    P.dB = ws<double>(c, "dB", N);
    P.dD = ws<double>(c, "dD", N);
    k_rho<<<nblocks(N), kT, 0, c->stream>>>(P.etap, P.A, P.rho, (int)N);
    LAUNCHCHK(c);
    const int nc = nrhs + 1;
    double2* rec0 = ws<double2>(c, "rec0", (size_t)N * (nc + 1));
    k_weights<<<dim3((unsigned)P.m1, (unsigned)nrhs), kT, 0, c->stream>>>(
        P.eta, P.rho, gam, nullptr, nullptr, nullptr, rec0, (int)N, (int)P.n, (int)P.m1, nc + 1, 1, 1, nullptr);
    LAUNCHCHK(c);
    CauchyPlan plan0 = plan_cauchy(N, nc, c->num_cu);
    double2* parts0 = ws<double2>(c, "parts0", (size_t)plan0.splits * nc * N);
    cauchy(c, rec0, N, nc, plan0, parts0);
    k_diag_fbie<<<nblocks(N), kT, 0, c->stream>>>(parts0, plan0.splits, nc, P.A, (int)N, two_n, P.dB, P.dD);
    LAUNCHCHK(c);
    // b = -y = -(D - diag(D1) + Lhat) gamma
    double* b = ws<double>(c, "rhs", (size_t)N * nrhs);
    dim3 ge(nblocks(N), (unsigned)nrhs);
    k_epilogue<<<ge, kT, 0, c->stream>>>(parts0, plan0.splits, nc, 1, gam, P.A, P.dD, 0.0, 1.0, 0.0, two_n,
                                         nullptr, (int)P.n, (int)P.m1, nullptr, b, (int)N);
    LAUNCHCHK(c);
    ensure_twiddles(c, P);
    HIPCHK(c, launch_circulant(gam, b, P.m1, P.n, nrhs, -1.0, P.tw, c->stream));
    // (2I + diag(B1) - B) mu = b
    if (o.prec == GNK_MIXED) setup_mixed(c, P);
    GmresOut g = gmres(c, P, GNK_OP_FB, b, nrhs, o, mu, o.prec == GNK_MIXED);
    if (h) {
      // h = [(D - diag(D1) + Lhat) mu - (2I + diag(B1) - B) gamma] / 2, f_B(gamma) from the first launch
      double* fbg = ws<double>(c, "fbg", (size_t)N * nrhs);
      k_epilogue<<<ge, kT, 0, c->stream>>>(parts0, plan0.splits, nc, 1, gam, P.A, P.dB, 2.0, 1.0, two_n, 0.0,
                                           nullptr, (int)P.n, (int)P.m1, nullptr, fbg, (int)N);
      LAUNCHCHK(c);
      apply_op(c, P, GNK_OP_FC, mu, nrhs, h);
      k_axpby<<<nblocks(N * nrhs), kT, 0, c->stream>>>(-0.5, fbg, 0.5, h, N * nrhs);
      LAUNCHCHK(c);
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info)
      for (int r = 0; r < nrhs; ++r) info[r] = g.info[r];
    return g.all_converged ? GNK_OK : GNK_NOT_CONVERGED;
  });
}

gnk_status gnk_fbie_ad(gnk_ctx* c, const gnk_domain* d, const double* gam, int nrhs, const gnk_opts* opts, double* mu,
                       gnk_info* info) {
  return guarded(c, [&]() -> gnk_status {
    check_domain(c, d, true);
    if (!gam || !mu || nrhs < 1 || nrhs > 1024 || mu == gam) {
      set_err(c, "bad arguments to gnk_fbie_ad");
      throw Fail{GNK_ERR_ARG};
    }
    gnk_opts o = resolve_opts(c, opts);
    Prep P = make_prep(c, d, true);
    validate_inputs(c, P, true, gam, nrhs);
    setup_fbiead(c, P);
    if (o.prec == GNK_MIXED) setup_mixed(c, P);
    GmresOut g = gmres(c, P, GNK_OP_GB, gam, nrhs, o, mu, o.prec == GNK_MIXED);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info)
      for (int r = 0; r < nrhs; ++r) info[r] = g.info[r];
    return g.all_converged ? GNK_OK : GNK_NOT_CONVERGED;
  });
}

}  // extern "C"

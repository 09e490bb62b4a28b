// Host driver of libgnk: context and workspace, batches of domains, input
// validation, operator application, the device-resident restarted GMRES, the
// launch-shape autotuner, and the C ABI entry points declared in include/gnk.h.
//
// Method (paper Sec. 3 and 4):
//   FBIE   : y = (D - diag(D1) + Lhat) gamma; solve (2I + diag(B1) - B) mu = -y;
//            h = [(D - diag(D1) + Lhat) mu - (2I + diag(B1) - B) gamma] / 2.
//   FBIEad : e from eq. (e:bve); solve (diag(e) + B^T + Phat) mu = gamma.
// Every product with B, D, B^T, D^T is one Cauchy sum S = E w followed by a
// per-node epilogue; the circulant blocks use the LDS FFT kernel.
//
// Every call works on a batch: one or more domains, each with its own columns
// (right-hand sides). A single-domain call is a batch of one whose flat
// vectors are the caller's arrays.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "gnk_internal.h"
#include "vec_kernels.inl"

// Scratch of gnk_cauchy_sum_noalloc: that entry point's workspace lives in
// this fixed device array (one copy per GPU, held until the process ends)
// instead of allocations. Host code uses only the address from
// hipGetSymbolAddress (gnk_ctx::scratch, taken once per device at
// gnk_create), never the array's name.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

struct gnk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;       // stream of all work (the caller's, or own_stream)
  hipStream_t own_stream = nullptr;   // blocking, default priority: capturable into graphs
  bool graphs = true;                 // replay the Arnoldi step from a captured hipGraph
  // instantiated Arnoldi-step graphs (FP64, mixed), kept across solves: each
  // solve captures its step and refreshes these with hipGraphExecUpdate, which
  // avoids a new instantiation when only kernel arguments changed
  hipGraphExec_t step_exec[6] = {};   // [mixed + 2 log2(steps)], 1, 2 or 4 steps
  // every value a cached step graph's launches take (see step_signature);
  // empty when the graph must be captured again
  std::vector<uint64_t> step_sig[6];
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
  std::map<int64_t, int> tw_ready;       // n -> 1 when the circulant table "tw<n>" is filled
  // pipelined convergence read-back of the GMRES iterations
  int* pinned = nullptr;                 // host-pinned, one int per Arnoldi step
  double* pinned_rel = nullptr;          // host-pinned residual estimates (mixed switch)
  size_t pinned_rel_n = 0;
  std::vector<hipEvent_t> step_ev;       // one event per Arnoldi step
  int* vflags = nullptr;                 // host-pinned input-check flags
  hipEvent_t val_ev = nullptr;           // recorded after the input checks
  // optional timing of the Cauchy-sum launches (HIP events on the context stream)
  bool prof = false;
  struct ProfRec {
    hipEvent_t a, b;
    double pair_cols, flops, pairs1;
    bool mixed, single;
    double tree_flops = 0.0;   // treecode products: the work of their lists
    bool tree = false;
    double fft_bytes = 0.0;    // circulant products (kept out of the pair totals)
    bool fft = false;
    bool spec = false;         // a fully masked speculative Arnoldi step: no work, not counted
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  gnk_prof prof_acc{};
  // autotuner results: key -> "tpt chunk"
  std::map<std::string, std::string> tune;
  bool tune_loaded = false;
  // host copies of uploaded tables stay alive until the next call
  std::vector<std::vector<char>> host_keep;
  // last contents uploaded to each named table: an unchanged table is not copied again
  std::map<std::string, std::pair<void*, std::vector<char>>> up_last;
  // host-mapped pinned memory that small kernels fill with results the host
  // reads after a stream synchronisation (flags, live count, per-column info)
  char* hostio = nullptr;
  size_t hostio_bytes = 0;
  // device address of this device's scratch array (gnk_cauchy_sum_noalloc), or null
  char* scratch = nullptr;
  // while set, ws() carves buffers from this region instead of allocating
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
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
  if (c->arena) {   // an entry point that allocates nothing: bump allocation in its scratch
    const size_t off = (c->arena_used + 255) & ~(size_t)255;
    if (off + bytes > c->arena_cap) {
      set_err(c, "input too large for the fixed scratch of %zu bytes: buffer '%s' needs %zu bytes at offset %zu "
              "(use the allocating entry point for this size)", c->arena_cap, name.c_str(), bytes, off);
      throw Fail{GNK_ERR_ARG};
    }
    c->arena_used = off + bytes;
    return reinterpret_cast<T*>(c->arena + off);
  }
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

// copy a host vector to a named device buffer (the host copy is kept alive
// until the next call, so the asynchronous copy may still read it)
template <class T>
T* upload(gnk_ctx* c, const std::string& name, const std::vector<T>& v) {
  T* d = ws<T>(c, name, std::max<size_t>(v.size(), 1));
  if (!v.empty() && c->arena) {   // scratch contents belong to no call: always copy
    std::vector<char> keep(sizeof(T) * v.size());
    memcpy(keep.data(), v.data(), keep.size());
    c->host_keep.push_back(std::move(keep));
    HIPCHK(c, hipMemcpyAsync(d, c->host_keep.back().data(), sizeof(T) * v.size(), hipMemcpyHostToDevice,
                             c->stream));
    return d;
  }
  if (!v.empty()) {
    auto& last = c->up_last[name];
    const size_t nb = sizeof(T) * v.size();
    if (last.first == (void*)d && last.second.size() == nb && memcmp(last.second.data(), v.data(), nb) == 0)
      return d;   // the device table already holds these contents
    last.first = nullptr;   // set again once the copy is enqueued
    std::vector<char> keep(sizeof(T) * v.size());
    memcpy(keep.data(), v.data(), keep.size());
    c->host_keep.push_back(std::move(keep));
    HIPCHK(c, hipMemcpyAsync(d, c->host_keep.back().data(), sizeof(T) * v.size(), hipMemcpyHostToDevice,
                             c->stream));
    last.first = d;
    last.second.assign(reinterpret_cast<const char*>(v.data()), reinterpret_cast<const char*>(v.data()) + nb);
  }
  return d;
}

// host-mapped pinned buffer of at least `bytes` (host pointer; the device
// pointer comes from hostio_dev). Grown only between uses: every call ends
// synchronised, and each use waits for its kernel before reading.
char* hostio(gnk_ctx* c, size_t bytes) {
  bytes = std::max<size_t>(bytes, 4096);
  if (c->hostio_bytes < bytes) {
    if (c->hostio) HIPCHK(c, hipHostFree(c->hostio));
    c->hostio = nullptr;
    c->hostio_bytes = 0;
    HIPCHK(c, hipHostMalloc((void**)&c->hostio, bytes, 0));
    c->hostio_bytes = bytes;
  }
  return c->hostio;
}
template <class T>
T* hostio_dev(gnk_ctx* c, T* host) {
  void* d = nullptr;
  HIPCHK(c, hipHostGetDevicePointer(&d, host, 0));
  return static_cast<T*>(d);
}

unsigned nblocks(int64_t n, int t = kT) { return (unsigned)((n + t - 1) / t); }

int64_t slots_of(const gnk_ctx* c) { return (int64_t)c->num_cu * 4 * 8; }   // 4 SIMDs x 8 waves

// ------------------------------------------------------------------ batches
// (lead, data) = (0,1), (1,1), (1,0); P_GM_MIXED: the P_GM columns grouped for
// mixed products (remainders of 3-7 columns padded to an 8-column group)
enum Pattern { P_GM = 0, P_SETUP = 1, P_LEAD = 2, P_GM_MIXED = 3 };
constexpr int kLead[4] = {0, 1, 1, 0};
constexpr int kData[4] = {1, 1, 0, 1};
constexpr int kWidths[4] = {8, 4, 2, 1};

struct PairShape {
  int tpt = 1;
  int chunk = 0;        // sources per workgroup (0: single-domain plan)
};

struct Batch {
  int ndom = 0, ncol = 0, maxN = 0, maxm1 = 0;
  int64_t T = 0;        // flat vector length
  std::vector<DomDev> dom;
  std::vector<ColDev> col;
  DomDev* d_dom = nullptr;
  ColDev* d_col = nullptr;
  PairShape shape;
  bool mixed = false;
  bool adjoint = false;
  bool second = false;   // eta'' and A' present (adjoint or no-subtraction operators)
  struct ItemSet {
    int4* d[4] = {nullptr, nullptr, nullptr, nullptr};
    int cnt[4] = {0, 0, 0, 0};
    double pair_cols = 0, flops = 0, pairs1 = 0;
    bool built = false;
  } sets[4];
  struct Circ {
    int64_t n;
    int64_t* offs;
    int nvec;
    double2* tw;
  };
  std::vector<Circ> circ;
  bool circ_built = false;
  // treecode far field (one domain, FP64), see build_tree
  struct Tree {
    bool on = false;
    int p = 0, levels = 0, nbox = 0, splits = 0, tiles = 0;
    std::vector<int> off, nb;
    double4* bounds = nullptr;
    double2* mom = nullptr;
    int* seg = nullptr;
    int* list = nullptr;
    size_t list_len = 0;
    double flops = 0.0;   // per column: 8 p_e + 8 per (target, far box), 16 per near pair
    int* perm = nullptr;  // level-0 slot -> leaf (device), and leaf -> slot
    int* invp = nullptr;
    bool ext = false;     // targets are the points tz (no j != i window), not the nodes
  } tree;
};

void check_domain(gnk_ctx* c, const gnk_domain* d, bool adjoint, bool second = false) {
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
  if (second && (!d->etapp || !d->Ap)) {
    set_err(c, "the equations without singularity subtraction need etapp and Ap");
    throw Fail{GNK_ERR_ARG};
  }
}

// Single-domain split plan: among the split counts whose waves fill whole
// rounds of the wave slots of the pair-kernel variant best (within 1% of the
// best fill), the fewest that give two rounds, else the most rounds; at least
// 128 sources per workgroup, at most 64 splits. Workgroups take unequal times
// (near source tiles cost more than far ones) and a second round lets the
// dispatcher even that out; more rounds shorten the products a little more
// but every split adds partial sums that the consumer has to read (measured
// at N = 17408: 123 us per product at 15 splits, 118 us at 30, 115 us at 45,
// with the reading growing by about 0.3 us per split).
int64_t single_max_splits(int64_t N) { return std::max<int64_t>(1, std::min<int64_t>(64, N / 128)); }
// Nt targets against Ns sources (the nodes, or separate points for the Cauchy
// integral at interior points)
void plan_pairs(gnk_ctx* c, int64_t Nt, int64_t Ns, int align, int width, bool mixed, int* tpt, int* chunk,
                int* splits) {
  int t = ((Nt + 127) / 128) * 64 >= slots_of(c) ? 2 : 1;
  if (const char* s = getenv("GNK_CAUCHY_TPT")) t = atoi(s) == 2 ? 2 : 1;
  // wave slots of the variant that runs the products (its register use sets
  // how many workgroups fit on a CU)
  const int64_t slots = (int64_t)c->num_cu * 4 * pairs_blocks_per_cu(width, t, mixed);
  const int64_t tiles = (Nt + 64 * t - 1) / (64 * t);
  const int64_t max_s = single_max_splits(Ns);
  std::vector<double> score((size_t)max_s + 1, 0.0), rounds((size_t)max_s + 1, 0.0);
  double best = 0.0;
  for (int64_t s = 1; s <= max_s; ++s) {
    rounds[s] = (double)(tiles * s * 4) / (double)slots;
    score[s] = rounds[s] / std::ceil(rounds[s]) * std::min(1.0, rounds[s]);
    best = std::max(best, score[s]);
  }
  int64_t bs = 0;
  for (int64_t s = 1; s <= max_s && !bs; ++s)
    if (score[s] >= best - 0.01 && rounds[s] >= 1.9) bs = s;
  for (int64_t s = max_s; s >= 1 && !bs; --s)
    if (score[s] >= best - 0.01) bs = s;
  if (const char* s = getenv("GNK_CAUCHY_SPLITS")) bs = std::max(1, atoi(s));
  int64_t ch = (Ns + bs - 1) / bs;
  ch = (ch + align - 1) / align * align;
  *tpt = t;
  *chunk = (int)ch;
  *splits = (int)((Ns + ch - 1) / ch);
}
void plan_single(gnk_ctx* c, int64_t N, int align, int width, bool mixed, int* tpt, int* chunk, int* splits) {
  plan_pairs(c, N, N, align, width, mixed, tpt, chunk, splits);
}

// Builds the batch tables and workspace. doms: host array; ncols: columns per
// domain; col_off: flat offset of column 0 of each domain (the columns of a
// domain are contiguous, N_d apart).
void build_batch(gnk_ctx* c, Batch& B, int ndom, const gnk_domain* doms, const int* ncols,
                 const std::vector<int64_t>& col_off, int64_t T, bool adjoint, bool mixed, const PairShape& shape,
                 int64_t force_N = 0) {
  B = Batch();
  B.ndom = ndom;
  B.T = T;
  B.mixed = mixed;
  B.adjoint = adjoint;
  B.shape = shape;
  const int align = mixed ? 256 : 16;
  int64_t Ntot = 0, rec_total = 0, rec32_total = 0, far32_total = 0, part_total = 0, sb_total = 0, tb_total = 0,
          sbf_total = 0;
  B.dom.resize(ndom);
  int c0 = 0;
  for (int d = 0; d < ndom; ++d) {
    check_domain(c, &doms[d], adjoint);
    DomDev& D = B.dom[d];
    memset(&D, 0, sizeof D);
    D.eta = static_cast<const double2*>(doms[d].eta);
    D.etap = static_cast<const double2*>(doms[d].etap);
    D.etapp = static_cast<const double2*>(doms[d].etapp);
    D.A = static_cast<const double2*>(doms[d].A);
    D.Ap = static_cast<const double2*>(doms[d].Ap);
    D.N = force_N ? (int)force_N : (int)(doms[d].m1 * doms[d].n);
    D.n = (int)doms[d].n;
    D.m1 = (int)doms[d].m1;
    D.ncols = ncols[d];
    D.c0 = c0;
    D.c = doms[d].c;
    c0 += ncols[d];
    if (ndom == 1 && shape.chunk == 0) {
      int t, ch, sp;
      const int width = ncols[d] >= 8 ? 8 : (ncols[d] >= 4 ? 4 : (ncols[d] >= 2 ? 2 : 1));
      plan_single(c, D.N, align, width, mixed, &t, &ch, &sp);
      B.shape.tpt = t;
      D.chunk = ch;
      D.splits = sp;
    } else {
      int64_t ch = std::max(align, shape.chunk > 0 ? shape.chunk : 2048);
      ch = (ch + align - 1) / align * align;
      const int64_t Nr = ((int64_t)D.N + align - 1) / align * align;
      ch = std::min(ch, Nr);
      D.chunk = (int)ch;
      D.splits = (int)((D.N + ch - 1) / ch);
    }
    B.maxN = std::max(B.maxN, D.N);
    B.maxm1 = std::max(B.maxm1, D.m1);
    Ntot += D.N;
    rec_total += (int64_t)D.N * rec_stride(D.ncols + 1);   // head, w.., b.. with a lead column
    rec32_total += (int64_t)D.N * rec32_stride(D.ncols + 1);
    far32_total += far32_size(D.N, D.ncols + 1);
    part_total += (int64_t)D.splits * (D.ncols + 1) * D.N;
    sb_total += (D.N + 63) / 64;
    tb_total += (D.N + 63) / 64;
    sbf_total += (D.N + kFarTile - 1) / kFarTile;
  }
  B.ncol = c0;
  double2* rho = ws<double2>(c, "b_rho", Ntot);
  double* dB = ws<double>(c, "b_dB", Ntot);
  double* dD = ws<double>(c, "b_dD", Ntot);
  double* ev = adjoint ? ws<double>(c, "b_e", Ntot) : nullptr;
  double* bu = ws<double>(c, "b_bu", Ntot);
  double2* rec = ws<double2>(c, "b_rec", rec_total);
  float2* rec32 = mixed ? ws<float2>(c, "b_rec32", rec32_total) : nullptr;
  float2* far32 = mixed ? ws<float2>(c, "b_far32", far32_total) : nullptr;
  double2* parts = ws<double2>(c, "b_parts", part_total);
  // tile bounds: far-tile classification (both precisions) and tile-relative records
  double4* sb = ws<double4>(c, "b_sb", sb_total);
  double4* tb = ws<double4>(c, "b_tb", tb_total);
  double4* sbf = ws<double4>(c, "b_sbf", sbf_total);
  double theta = 1.0;
  if (const char* e = getenv("GNK_MIXED_THETA")) theta = atof(e);
  int64_t on = 0, orc = 0, orc32 = 0, ofar = 0, op = 0, osb = 0, otb = 0, osbf = 0;
  for (int d = 0; d < ndom; ++d) {
    DomDev& D = B.dom[d];
    D.rho = rho + on;
    D.dB = dB + on;
    D.dD = dD + on;
    D.e = ev ? ev + on : nullptr;
    D.bu = bu + on;
    D.rec = rec + orc;
    D.rec32 = rec32 ? rec32 + orc32 : nullptr;
    D.far32 = far32 ? far32 + ofar : nullptr;
    D.parts = parts + op;
    D.sb = sb ? sb + osb : nullptr;
    D.tb = tb ? tb + otb : nullptr;
    D.sbf = sbf + osbf;
    D.far2 = (1.0 + theta) * (1.0 + theta);
    // The FP64 far form sums conj(z') w m - b m about the source tile's centre
    // (exact algebra); separation only bounds how much rounding the two terms'
    // cancellation and the expanded |z' - v|^2 amplify: (2 + t)/t and its
    // square for separation (1 + t)(r_t + r_s), 25 at t = 0.5.
    D.far2d = 2.25;
    on += D.N;
    orc += (int64_t)D.N * rec_stride(D.ncols + 1);
    orc32 += (int64_t)D.N * rec32_stride(D.ncols + 1);
    ofar += far32_size(D.N, D.ncols + 1);
    op += (int64_t)D.splits * (D.ncols + 1) * D.N;
    osb += (D.N + 63) / 64;
    otb += (D.N + 63) / 64;
    osbf += (D.N + kFarTile - 1) / kFarTile;
    for (int r = 0; r < D.ncols; ++r) B.col.push_back(ColDev{d, r, col_off[d] + (int64_t)r * D.N});
  }
  B.d_dom = upload(c, "b_dom", B.dom);
  B.d_col = upload(c, "b_col", B.col);
  HIPCHK(c, launch_node_tile_bounds(B.d_dom, ndom, B.maxN, B.shape.tpt, c->stream));
}

// Work items of a pattern: every domain (largest first), column group, target
// tile and source split; grouped by column-group width.
void build_items(gnk_ctx* c, Batch& B, int p) {
  auto& S = B.sets[p];
  if (S.built) return;
  const int lead = kLead[p], data = kData[p];
  std::vector<int> order(B.ndom);
  for (int d = 0; d < B.ndom; ++d) order[d] = d;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return B.dom[a].N > B.dom[b].N; });
  std::vector<int4> lists[4];
  S.pair_cols = S.flops = S.pairs1 = 0;
  for (int d : order) {
    const DomDev& D = B.dom[d];
    const int wcols = lead + data * D.ncols;
    const int tile = 64 * B.shape.tpt;
    const int NT = D.tz ? D.Nt : D.N;   // targets: separate points, or the nodes
    const int tiles = (NT + tile - 1) / tile;
    const double pairs = D.tz ? (double)NT * (double)D.N : (double)D.N * (double)(D.N - 1);
    S.pair_cols += pairs * wcols;
    S.flops += pairs * (16.0 + 8.0 * (wcols - 1));
    if (wcols == 1) S.pairs1 += pairs;
    int r0 = 0;
    while (r0 < wcols) {
      int wi = 3;
      for (int k = 0; k < 4; ++k)
        if (kWidths[k] <= wcols - r0) {
          wi = k;
          break;
        }
      int w = kWidths[wi];
      int code = r0;
      if (p == P_GM_MIXED && wcols - r0 >= 3 && wcols - r0 < 8) {
        // padded 8-column group of the remaining columns (width in bits 20..)
        wi = 0;
        w = wcols - r0;
        code = r0 | (w << 20);
      }
      // Records larger than half an XCD's L2 (4 MB): split-major, so the
      // workgroups resident together read one source range (measured at
      // N = 133120: 28% shorter products than tile-major). Smaller ones stay
      // in L2 either way and go tile-major, whose last round is cheaper
      // (3% at N = 17408).
      if ((int64_t)D.N * rec_stride(wcols) * (int64_t)sizeof(double2) > (int64_t)2 << 20) {
        for (int g = 0; g < D.splits; ++g)
          for (int t = 0; t < tiles; ++t) lists[wi].push_back(make_int4(d, t, g, code));
      } else if (D.tz) {
        for (int t = 0; t < tiles; ++t)
          for (int g = 0; g < D.splits; ++g) lists[wi].push_back(make_int4(d, t, g, code));
      } else {
        // the items whose source range meets the target tile's own component
        // (mostly near tiles, the costliest) go first, so that the cheap ones
        // fill the end of the launch
        std::vector<int4> rest;
        for (int t = 0; t < tiles; ++t) {
          const int64_t c0 = (int64_t)(t * tile / D.n) * D.n;
          const int64_t c1 = std::min<int64_t>(D.N, ((int64_t)(std::min(D.N, (t + 1) * tile) - 1) / D.n + 1) * D.n);
          for (int g = 0; g < D.splits; ++g) {
            const int64_t a0 = (int64_t)g * D.chunk, a1 = std::min<int64_t>(D.N, a0 + D.chunk);
            (std::max(a0, c0) < std::min(a1, c1) ? lists[wi] : rest).push_back(make_int4(d, t, g, code));
          }
        }
        lists[wi].insert(lists[wi].end(), rest.begin(), rest.end());
      }
      r0 += w;
    }
  }
  for (int k = 0; k < 4; ++k) {
    S.cnt[k] = (int)lists[k].size();
    S.d[k] = upload(c, "b_items" + std::to_string(p) + "_" + std::to_string(k), lists[k]);
  }
  S.built = true;
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

// ----------------------------------------------------------------- treecode
// Far-field compression for one domain (the treecode of csrc/tree.hip): box
// bounds on the device, then on the host one depth-first pass per target
// tile over the box hierarchy: a box whose bounding circle is separated from
// the tile's by (1 + theta)(r_t + r_b) is far (its expansion), a leaf that is
// not is near (its four 64-node blocks, summed directly); each tile's list is
// cut into 4 splits ranges of about equal estimated cost (far box 4p_e + 24,
// near source 13 per target, the tile's own window 16). theta = 1.5 bounds
// r_b/|z - c_b| by 0.4, so p = log(far_tol)/log(0.4) terms meet far_tol for
// every far box; each (tile, box) entry takes the p_e its own ratio
// rho_e = r_b/(|c_t - c_b| - r_t) >= r_b/|z - c_b| needs, which keeps the bound.
constexpr double kTreeTheta = 1.5;

int tree_terms(double far_tol) {
  const double rho = 1.0 / (1.0 + kTreeTheta);
  const int p = (int)std::ceil(std::log(far_tol) / std::log(rho));
  return std::max(4, std::min(kTreeMaxP, p));
}

// perm: the indices of pts in the order of their positions along a Hilbert
// curve (16 bits per coordinate over the points' bounding square; ties keep
// index order). The curve has no jumps, so any run of consecutive indices
// lies in a compact region of the plane.
void hilbert_order(const std::vector<double2>& pts, std::vector<int>& perm) {
  const size_t n = pts.size();
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (const auto& p : pts) {
    x0 = std::min(x0, p.x), x1 = std::max(x1, p.x), y0 = std::min(y0, p.y), y1 = std::max(y1, p.y);
  }
  const double span = std::max(x1 - x0, y1 - y0);
  const double sc = span > 0.0 ? 65535.0 / span : 0.0;
  constexpr uint32_t side = 1u << 16;
  auto distance = [](uint32_t x, uint32_t y) {   // position along the curve of cell (x, y)
    uint64_t d = 0;
    for (uint32_t h = side / 2; h > 0; h /= 2) {
      const uint32_t rx = (x & h) ? 1u : 0u, ry = (y & h) ? 1u : 0u;
      d += (uint64_t)h * h * ((3u * rx) ^ ry);
      if (ry == 0) {   // rotate the quadrant
        if (rx == 1) {
          x = side - 1 - x;
          y = side - 1 - y;
        }
        std::swap(x, y);
      }
    }
    return d;
  };
  std::vector<uint64_t> code(n);
  perm.resize(n);
  for (size_t b = 0; b < n; ++b) {
    const uint32_t qx = (uint32_t)std::min(65535.0, std::max(0.0, (pts[b].x - x0) * sc));
    const uint32_t qy = (uint32_t)std::min(65535.0, std::max(0.0, (pts[b].y - y0) * sc));
    code[b] = distance(qx, qy);
    perm[b] = (int)b;
  }
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return code[a] < code[b]; });
}

void build_tree(gnk_ctx* c, Batch& B, double far_tol, bool ext = false) {
  if (B.ndom != 1 || B.mixed) {
    set_err(c, "the treecode takes one domain in FP64");
    throw Fail{GNK_ERR_ARG};
  }
  DomDev& D = B.dom[0];
  auto& T = B.tree;
  const int N = D.N, tpt = B.shape.tpt, kt = 64 * tpt;
  const int NT = ext ? D.Nt : N;   // targets
  T = Batch::Tree{};
  T.ext = ext;
  T.p = tree_terms(far_tol);
  int total = 0;
  // far entries carry the box index in 24 bits
  if ((int64_t)2 * ((N + kLeaf - 1) / kLeaf) + 64 >= ((int64_t)1 << 24)) {
    set_err(c, "the treecode takes at most about 2^31 nodes");
    throw Fail{GNK_ERR_ARG};
  }
  for (int nb = (N + kLeaf - 1) / kLeaf;; nb = (nb + 1) / 2) {
    T.off.push_back(total);
    T.nb.push_back(nb);
    total += nb;
    if (nb == 1) break;
  }
  T.levels = (int)T.nb.size();
  T.nbox = total;
  T.bounds = ws<double4>(c, "t_bounds", total);
  T.mom = ws<double2>(c, "t_mom", (size_t)total * T.p);
  double4* bbox = ws<double4>(c, "t_bbox", total);
  unsigned long long* rbits = ws<unsigned long long>(c, "t_rbits", total);
  // The leaves take the level-0 slots in the Hilbert order of their centres, so
  // that a box of 2^l slots is a compact cluster of the plane (in node order a
  // box could join boundary pieces far apart, and few boxes would be far).
  const int nleaf = T.nb[0];
  double4* lbox = ws<double4>(c, "t_lbox", nleaf);
  HIPCHK(c, launch_leaf_boxes(D.eta, N, nleaf, lbox, c->stream));
  std::vector<double4> hl((size_t)nleaf);
  HIPCHK(c, hipMemcpyAsync(hl.data(), lbox, sizeof(double4) * nleaf, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<double2> centre((size_t)nleaf);
  for (int b = 0; b < nleaf; ++b) centre[b] = make_double2(0.5 * (hl[b].x + hl[b].y), 0.5 * (hl[b].z + hl[b].w));
  std::vector<int> perm, invp((size_t)nleaf);
  hilbert_order(centre, perm);
  for (int s2 = 0; s2 < nleaf; ++s2) invp[perm[s2]] = s2;
  T.perm = upload(c, "t_perm", perm);
  T.invp = upload(c, "t_invp", invp);
  HIPCHK(c, launch_box_bounds(D.eta, N, T.off.data(), T.nb.data(), T.levels, lbox, T.perm, T.invp, bbox, rbits,
                              T.bounds, c->stream));
  T.tiles = (NT + kt - 1) / kt;
  std::vector<double4> hb(total), ht(T.tiles);
  HIPCHK(c, hipMemcpyAsync(hb.data(), T.bounds, sizeof(double4) * total, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(ht.data(), D.tb, sizeof(double4) * T.tiles, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // about two rounds of resident workgroups
  const int64_t resident = (int64_t)c->num_cu * 5;
  int S = (int)std::max<int64_t>(1, std::min<int64_t>(16, (2 * resident + T.tiles - 1) / T.tiles));
  if (const char* e = getenv("GNK_TREE_SPLITS")) S = std::max(1, atoi(e));
  T.splits = S;
  const double f2 = (1.0 + kTreeTheta) * (1.0 + kTreeTheta);
  const double cnear = 13.0, cself = 16.0;
  // rho^k <= far_tol exactly when rho <= far_tol^(1/k): the order p_e of a far
  // entry is the least k >= 2 (at most p) whose threshold rho meets
  std::vector<double> thr((size_t)T.p + 1, 0.0);
  for (int k = 1; k <= T.p; ++k) thr[k] = std::pow(far_tol, 1.0 / k);
  std::vector<int> seg((size_t)T.tiles * (4 * S + 1));
  // the tiles' lists are independent: contiguous tile ranges on a few host
  // threads, each list local to its thread, then joined in tile order
  const int nth = std::max(1, std::min({16, (int)std::thread::hardware_concurrency(), (T.tiles + 63) / 64}));
  std::vector<std::vector<int>> part((size_t)nth);
  std::vector<char> failed((size_t)nth, 0);
  std::vector<double> work((size_t)nth, 0.0);
  auto lists_for = [&](int th) {
    const int t0 = (int)((int64_t)T.tiles * th / nth), t1 = (int)((int64_t)T.tiles * (th + 1) / nth);
    std::vector<int>& lst = part[(size_t)th];
    try {
      std::vector<int> ent;
      std::vector<double> cost;
      int stack[2 * 34][2];   // depth-first: at most one pending sibling per level
      for (int t = t0; t < t1; ++t) {
        ent.clear();
        cost.clear();
        const double4 tt = ht[t];
        const int base = t * kt, top = T.levels - 1;
        const double nt = (double)std::min(kt, NT - base);
        int sp = 0;
        for (int b = T.nb[top] - 1; b >= 0; --b) {
          stack[sp][0] = top;
          stack[sp][1] = b;
          ++sp;
        }
        while (sp > 0) {
          --sp;
          const int l = stack[sp][0], b = stack[sp][1];
          const double4 bb = hb[T.off[l] + b];
          const double dx = tt.x - bb.x, dy = tt.y - bb.y, rr = tt.z + bb.z;
          const double d2 = dx * dx + dy * dy;
          if (d2 > f2 * rr * rr) {
            const double rho = bb.z / (std::sqrt(d2) - tt.z);
            int pe = 2;
            while (pe < T.p && rho > thr[pe]) ++pe;
            ent.push_back((pe << 24) | (T.off[l] + b));
            cost.push_back(4.0 * pe + 24.0);
            work[(size_t)th] += nt * (8.0 * pe + 8.0);
          } else if (l == 0) {
            for (int k = 0; k < kLeaf / 64; ++k) {
              const int j0 = perm[b] * kLeaf + k * 64;
              if (j0 >= N) break;
              const int j1 = std::min(N, j0 + 64);
              const int ov = ext ? 0 : std::max(0, std::min(j1, base + kt) - std::max(j0, base));
              ent.push_back(~(j0 / 64));
              cost.push_back(cnear * (j1 - j0 - ov) + cself * ov);
              work[(size_t)th] += 16.0 * (nt * (j1 - j0) - ov);
            }
          } else {
            // children pushed in reverse so that the list keeps slot order
            if (2 * b + 1 < T.nb[l - 1]) {
              stack[sp][0] = l - 1;
              stack[sp][1] = 2 * b + 1;
              ++sp;
            }
            stack[sp][0] = l - 1;
            stack[sp][1] = 2 * b;
            ++sp;
          }
        }
        double tot = 0.0;
        for (double x : cost) tot += x;
        int* sg = seg.data() + (size_t)t * (4 * S + 1);
        const int64_t start = (int64_t)lst.size();
        sg[0] = (int)start;
        double acc = 0.0;
        size_t e = 0;
        for (int k = 1; k < 4 * S; ++k) {
          const double target = tot * k / (4.0 * S);
          while (e < ent.size() && acc + 0.5 * cost[e] < target) acc += cost[e++];
          sg[k] = (int)(start + (int64_t)e);
        }
        sg[4 * S] = (int)(start + (int64_t)ent.size());
        if (lst.size() + ent.size() > (size_t)INT32_MAX / 2) {
          failed[(size_t)th] = 1;   // reported after the join
          return;
        }
        lst.insert(lst.end(), ent.begin(), ent.end());
      }
    } catch (...) {
      failed[(size_t)th] = 1;
    }
  };
  {
    std::vector<std::thread> pool;
    int spawned = 1;
    try {
      for (; spawned < nth; ++spawned) pool.emplace_back(lists_for, spawned);
    } catch (...) {
    }
    for (int th = spawned; th < nth; ++th) lists_for(th);   // ranges that got no thread
    lists_for(0);
    for (auto& t : pool) t.join();
  }
  size_t len = 0;
  bool cut = false;
  T.flops = 0.0;
  for (int th = 0; th < nth; ++th) {
    T.flops += work[(size_t)th];
    len += part[(size_t)th].size();
    cut = cut || failed[(size_t)th];
  }
  if (cut || len > (size_t)INT32_MAX / 2) {
    set_err(c, "treecode interaction lists too long");
    throw Fail{GNK_ERR_OOM};
  }
  std::vector<int> list;
  list.reserve(len);
  for (int th = 0; th < nth; ++th) {
    const int t0 = (int)((int64_t)T.tiles * th / nth), t1 = (int)((int64_t)T.tiles * (th + 1) / nth);
    const int off = (int)list.size();
    for (int t = t0; t < t1; ++t)
      for (int k = 0; k <= 4 * S; ++k) seg[(size_t)t * (4 * S + 1) + k] += off;
    list.insert(list.end(), part[(size_t)th].begin(), part[(size_t)th].end());
  }
  T.list_len = list.size();
  T.list = upload(c, "t_list", list);
  T.seg = upload(c, "t_seg", seg);
  D.splits = S;
  D.chunk = N;
  D.parts = ws<double2>(c, "t_parts", (size_t)S * (D.ncols + 1) * NT);
  B.d_dom = upload(c, "b_dom", B.dom);
  T.on = true;
}

// the Cauchy sums of one pattern by the treecode, one weight column at a time
void tree_pairs(gnk_ctx* c, Batch& B, int p, const int* active) {
  auto& T = B.tree;
  const DomDev& D = B.dom[0];
  const int lead = kLead[p], wcols = lead + kData[p] * D.ncols;
  gnk_ctx::ProfRec pr{};
  if (c->prof) {
    // counted as the pairs the direct sum would take
    const double pairs = T.ext ? (double)D.N * (double)D.Nt : (double)D.N * (double)(D.N - 1);
    pr = gnk_ctx::ProfRec{pool_event(c), pool_event(c), pairs * wcols, pairs * (16.0 + 8.0 * (wcols - 1)),
                          wcols == 1 ? pairs : 0.0, false, wcols == 1, T.flops * wcols, true};
    HIPCHK(c, hipEventRecord(pr.a, c->stream));
  }
  for (int col = 0; col < wcols; ++col) {
    HIPCHK(c, launch_tree_moments(D.rec, rec_stride(wcols), kRecHead + col, D.N, T.bounds, T.perm, T.off.data(),
                                  T.nb.data(), T.levels, T.p, T.mom, c->stream));
    HIPCHK(c, launch_tree_eval(B.d_dom, T.tiles, B.shape.tpt, T.seg, T.list, T.bounds, T.mom, T.p, T.splits, col,
                               wcols, active, lead, T.ext, c->stream));
  }
  if (c->prof) {
    HIPCHK(c, hipEventRecord(pr.b, c->stream));
    c->prof_pending.push_back(pr);
  }
}

// threads of k_records32 for pattern p: one per node and weight column, the
// columns rounded up to a multiple of 8, for the largest domain of the batch
int64_t records32_threads(const Batch& B, int p) {
  int64_t t = 0;
  for (const DomDev& D : B.dom) {
    const int wc = kLead[p] + kData[p] * D.ncols;
    t = std::max(t, (int64_t)D.N * ((wc + 7) / 8 * 8));
  }
  return t;
}

// All Cauchy sums of a pattern for the batch (one launch per column-group width).
void pairs(gnk_ctx* c, Batch& B, int p, bool mixed, const int* active) {
  if (B.tree.on && !mixed) {
    tree_pairs(c, B, p, active);
    return;
  }
  if (mixed && p == P_GM) p = P_GM_MIXED;
  build_items(c, B, p);
  auto& S = B.sets[p];
  if (mixed) HIPCHK(c, launch_records32(B.d_dom, B.ndom, records32_threads(B, p), kLead[p], kData[p], c->stream));
  gnk_ctx::ProfRec pr{};
  if (c->prof) {
    pr = gnk_ctx::ProfRec{pool_event(c), pool_event(c), S.pair_cols, S.flops, S.pairs1, mixed,
                          S.pairs1 > 0 && S.pairs1 == S.pair_cols};
    HIPCHK(c, hipEventRecord(pr.a, c->stream));
  }
  for (int k = 0; k < 4; ++k) {
    if (!S.cnt[k]) continue;
    HIPCHK(c, launch_pairs(B.d_dom, S.d[k], S.cnt[k], kWidths[k], B.shape.tpt, kLead[p], kData[p], mixed,
                           B.dom[0].tz != nullptr, active, c->stream));
  }
  if (c->prof) {
    HIPCHK(c, hipEventRecord(pr.b, c->stream));
    c->prof_pending.push_back(pr);
  }
}

void build_circ(gnk_ctx* c, Batch& B) {
  if (B.circ_built) return;
  std::map<int64_t, std::vector<int64_t>> byn;
  for (const ColDev& C : B.col) {
    const DomDev& D = B.dom[C.d];
    for (int k = 0; k < D.m1; ++k) byn[D.n].push_back(C.off + (int64_t)k * D.n);
  }
  for (auto& kv : byn) {
    const int64_t n = kv.first;
    const std::string tn = "tw" + std::to_string(n);
    const size_t cnt = circulant_uses_fft(n) ? (size_t)n / 2 : (size_t)(n + 1) / 2;
    double2* tw = ws<double2>(c, tn, cnt + 1);
    if (!c->tw_ready[n]) {
      HIPCHK(c, launch_twiddles(tw, n, c->stream));
      c->tw_ready[n] = 1;
    }
    int64_t* offs = upload(c, "circ" + std::to_string(n), kv.second);
    B.circ.push_back(Batch::Circ{n, offs, (int)kv.second.size(), tw});
  }
  B.circ_built = true;
}

void circulant(gnk_ctx* c, Batch& B, const double* x, double* y, double sign) {
  build_circ(c, B);
  gnk_ctx::ProfRec pr{};
  if (c->prof) {
    double units = 0.0;
    for (auto& ci : B.circ) units += (double)ci.nvec * (double)ci.n;
    pr = gnk_ctx::ProfRec{pool_event(c), pool_event(c), 0.0, 0.0, 0.0, false, false, 0.0, false, 24.0 * units, true};
    HIPCHK(c, hipEventRecord(pr.a, c->stream));
  }
  std::vector<CircClass> cls;
  for (auto& ci : B.circ) cls.push_back(CircClass{ci.offs, ci.nvec, ci.n, ci.tw});
  HIPCHK(c, launch_circulant(x, y, cls.data(), (int)cls.size(), sign, c->stream));
  if (c->prof) {
    HIPCHK(c, hipEventRecord(pr.b, c->stream));
    c->prof_pending.push_back(pr);
  }
}

dim3 node_grid(const Batch& B) { return dim3(nblocks(B.maxN), (unsigned)B.ndom); }
dim3 col_grid(const Batch& B) { return dim3(nblocks(B.maxN), (unsigned)B.ncol); }

// Input checks on the device (finite values, A and, where the operator needs
// it, eta' nonzero). validate_enqueue queues them, writing their flags to
// host-mapped memory; validate_finish waits for that launch alone and throws
// on a failed check. Between the two a caller may queue work that writes only
// the library's workspace (the right-hand side product, diagonals), so that
// the wait overlaps it; nothing the caller owns is written before the finish,
// and an error return synchronises the stream first. (Every call ends
// synchronised, so no earlier check can still write the flags the host zeroes.)
void validate_enqueue(gnk_ctx* c, Batch& B, const double* x, int64_t len) {
  if (!c->vflags) HIPCHK(c, hipHostMalloc((void**)&c->vflags, 3 * sizeof(int), 0));
  if (!c->val_ev) HIPCHK(c, hipEventCreateWithFlags(&c->val_ev, hipEventDisableTiming));
  volatile int* fl = c->vflags;
  fl[0] = fl[1] = fl[2] = 0;
  if (!x) len = 0;
  const dim3 grid(std::max(nblocks(B.maxN), nblocks(std::max<int64_t>(len, 1))), (unsigned)B.ndom + 1);
  k_validate_inputs<<<grid, kT, 0, c->stream>>>(B.d_dom, B.ndom, (B.adjoint || B.second) ? 1 : 0, x, len,
                                                hostio_dev(c, c->vflags));
  LAUNCHCHK(c);
  HIPCHK(c, hipEventRecord(c->val_ev, c->stream));
}

void validate_finish(gnk_ctx* c) {
  HIPCHK(c, hipEventSynchronize(c->val_ev));
  const volatile int* fl = c->vflags;
  if (fl[0]) {
    set_err(c, "non-finite value in the inputs");
    throw Fail{GNK_ERR_NONFINITE};
  }
  if (fl[1]) {
    set_err(c, "A vanishes at a node");
    throw Fail{GNK_ERR_ZERO_A};
  }
  if (fl[2]) {
    set_err(c, "eta' vanishes at a node (the adjoint equation divides by eta')");
    throw Fail{GNK_ERR_ZERO_ETAP};
  }
}

void validate(gnk_ctx* c, Batch& B, const double* x, int64_t len) {
  validate_enqueue(c, B, x, len);
  validate_finish(c);
}

// rho, and diag(B1), diag(D1) from S = E(rho) (leading column only)
// the diagonal limit of N for the operators without singularity subtraction
void setup_ndiag(gnk_ctx* c, Batch& B) {
  k_ndiag<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom);
  LAUNCHCHK(c);
}

void setup_diag(gnk_ctx* c, Batch& B) {
  k_rho<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom);
  LAUNCHCHK(c);
  k_lead_records<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom, C_RHO);
  LAUNCHCHK(c);
  pairs(c, B, P_LEAD, false, nullptr);
  k_diag_fbie<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom, 1, 0);
  LAUNCHCHK(c);
}

// e of eq. (e:bve) from S = E eta'
void setup_evec(gnk_ctx* c, Batch& B) {
  k_lead_records<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom, C_ETAP);
  LAUNCHCHK(c);
  pairs(c, B, P_LEAD, false, nullptr);
  k_evec<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom);
  LAUNCHCHK(c);
}

// --------------------------------------------------------- operator product
// The operators as a record weight (cw: x times rho or A) and an epilogue
//   y = a0 x + dsign dg x + cI Im(Cout S) + cR Re(Cout S) (+ Phat x when mean)
struct OpForm {
  int cw = C_RHO, cout = C_A, dsel = D_NONE;
  double a0 = 0.0, dsign = 0.0, cI = 0.0, cR = 0.0;
  bool mean = false;
};

OpForm op_form(gnk_ctx* c, int op) {
  OpForm f;
  switch (op) {
    case GNK_OP_FB:   // 2x + diag(B1) x - B x,  B x = -(2/n) Im(A E(rho x))
      f.cw = C_RHO; f.cout = C_A; f.a0 = 2.0; f.dsel = D_B; f.dsign = 1.0; f.cI = 1.0; break;
    case GNK_OP_FC:   // D x - diag(D1) x (+ Lhat x),  D x = -(2/n) Re(A E(rho x))
      f.cw = C_RHO; f.cout = C_A; f.dsel = D_D; f.dsign = -1.0; f.cR = -1.0; break;
    case GNK_OP_GB:   // e x + B^T x + Phat x,  B^T x = (2/n) Im(rho E(A x))
      f.cw = C_A; f.cout = C_RHO; f.dsel = D_E; f.dsign = 1.0; f.cI = 1.0; f.mean = true; break;
    case GNK_OP_FB_T: // 2x + diag(B1) x - B^T x
      f.cw = C_A; f.cout = C_RHO; f.a0 = 2.0; f.dsel = D_B; f.dsign = 1.0; f.cI = -1.0; break;
    case GNK_OP_FC_T: // D^T x - diag(D1) x - Lhat x,  D^T x = (2/n) Re(rho E(A x))
      f.cw = C_A; f.cout = C_RHO; f.dsel = D_D; f.dsign = -1.0; f.cR = 1.0; break;
    case GNK_OP_GB_T: // e x + B x + Phat x
      f.cw = C_RHO; f.cout = C_A; f.dsel = D_E; f.dsign = 1.0; f.cI = -1.0; f.mean = true; break;
    case GNK_OP_FB_U: // x - B x - Nd x  (no subtraction)
      f.cw = C_RHO; f.cout = C_A; f.a0 = 1.0; f.dsel = D_BU; f.dsign = -1.0; f.cI = 1.0; break;
    case GNK_OP_GB_U: // x + B^T x + Nd x + Phat x  (no subtraction)
      f.cw = C_A; f.cout = C_RHO; f.a0 = 1.0; f.dsel = D_BU; f.dsign = 1.0; f.cI = 1.0; f.mean = true; break;
    default:
      set_err(c, "unknown operator %d", op);
      throw Fail{GNK_ERR_ARG};
  }
  return f;
}

// y = op(x) for every column of the batch; active: optional mask.
struct ApplyArgs {
  const int* active = nullptr;
  bool mixed = false;        // FP32 far tiles (batch built with mixed records)
  // the partial sums of E(w x) from the last pair launch are those this
  // operator needs (same weights and x): apply only the epilogue
  bool reuse_sums = false;
};

void apply_op(gnk_ctx* c, Batch& B, int op, const double* x, double* y, const ApplyArgs& a = {}) {
  if (op == GNK_OP_LHAT) {
    k_axpby<<<nblocks(B.T), kT, 0, c->stream>>>(0.0, x, 0.0, y, B.T);
    LAUNCHCHK(c);
    circulant(c, B, x, y, 1.0);
    return;
  }
  const OpForm f = op_form(c, op);
  const int M = B.maxm1;
  double* mean = f.mean ? ws<double>(c, "mean", (size_t)B.ncol * M) : nullptr;
  if (a.reuse_sums && f.mean) {
    set_err(c, "internal: reused sums need a plain product of x");
    throw Fail{GNK_ERR_ARG};
  }
  if (!a.reuse_sums) {
    k_weights<<<dim3((unsigned)B.maxm1, (unsigned)B.ncol), kT, 0, c->stream>>>(B.d_dom, B.d_col, f.cw, x, a.active,
                                                                               0, mean, M);
    LAUNCHCHK(c);
    pairs(c, B, P_GM, a.mixed, a.active);
  }
  k_epilogue<<<col_grid(B), kT, 0, c->stream>>>(B.d_dom, B.d_col, x, f.cout, f.dsel, f.a0, f.dsign, f.cI, f.cR, mean,
                                                M, a.active, 0, y);
  LAUNCHCHK(c);
  if (op == GNK_OP_FC || op == GNK_OP_FC_T) circulant(c, B, x, y, op == GNK_OP_FC ? 1.0 : -1.0);
}

// ------------------------------------------------------------------ GMRES
struct GmresOut {
  std::vector<gnk_info> info;
  bool all_converged = false;
  // the last pair launch was the FP64 residual product of the returned x for
  // every column, with the weights rho x (FB, FB_U): D.parts hold E(rho x)
  bool sums_of_x = false;
};

// Restarted GMRES on every column of the batch (x, b: flat). With `mixed`,
// the Arnoldi products switch to the mixed-precision pair kernel once the
// residual estimate of every column is below o.inner_tol (relaxed products:
// an error of relative size e in a product made when the residual is r
// perturbs the final residual by about e*r, so FP32 far tiles are harmless
// once r <= tol / e). The residual that starts every cycle is always
// recomputed with FP64 products, so each restart is a step of FP64 iterative
// refinement.
GmresOut gmres(gnk_ctx* c, Batch& B, int op, const double* b, const gnk_opts& o, double* x, bool mixed = false) {
  const ApplyArgs am;   // FP64 products for every true residual
  const int ncol = B.ncol;
  const int64_t T = B.T;
  const int restart = o.restart;
  const int ldp = restart + 1;
  // vector-kernel blocking: 256..kMaxChunk elements per block, about 256
  // blocks per column of the largest domain, or fewer per column when the
  // batch's columns give more than about 8192 blocks together (each block
  // sums its column's block partials, so fewer blocks per column also means
  // less of that)
  const int per_blk = (int)std::max<int64_t>(
      kT, std::min<int64_t>(kMaxChunk, std::max<int64_t>(((int64_t)B.maxN + 255) / 256, (T + 8191) / 8192)));
  const int nblk = (B.maxN + per_blk - 1) / per_blk;

  double* V = ws<double>(c, "V", (size_t)(restart + 1) * T);
  double* P1 = ws<double>(c, "gmP1", (size_t)ncol * nblk * ldp);
  double* P2 = ws<double>(c, "gmP2", (size_t)ncol * nblk * ldp);
  GmresState st;
  st.ldh = restart + 1;
  st.hstride = st.ldh * restart;
  double* dbl = ws<double>(c, "gmdbl", (size_t)ncol * (4 + st.hstride + 2 * kMaxRestart + (kMaxRestart + 1) +
                                                     kMaxRestart));
  int* ints = ws<int>(c, "gmint", (size_t)ncol * 5 + 4);
  {
    double* q = dbl;
    st.bnorm = q; q += ncol;
    st.true_relres = q; q += ncol;
    st.relres = q; q += ncol;
    st.invbeta = q; q += ncol;
    st.H = q; q += (size_t)ncol * st.hstride;
    st.cs = q; q += (size_t)ncol * kMaxRestart;
    st.sn = q; q += (size_t)ncol * kMaxRestart;
    st.g = q; q += (size_t)ncol * (kMaxRestart + 1);
    st.y = q;
    int* r = ints;
    st.active = r; r += ncol;
    st.converged = r; r += ncol;
    st.kdim = r; r += ncol;
    st.inner_it = r; r += ncol;
    st.live = r;
    st.step = r + 1;
    st.done = r + 2;
  }
  // the step index of odd steps (see k_gs_finish)
  int* const step_odd = ints + (size_t)ncol * 5 + 3;
  // component sums of the Arnoldi vectors for operators with Phat: S slots
  // per block (a chunk of per_blk entries meets at most (per_blk-1)/n + 2
  // components)
  if (op == GNK_OP_FC || op == GNK_OP_FC_T || op == GNK_OP_LHAT) {
    set_err(c, "internal: the Arnoldi step has no circulant part (operator %d)", op);
    throw Fail{GNK_ERR_ARG};
  }
  const OpForm form = op_form(c, op);
  int nmin = B.dom[0].n;
  for (const DomDev& D : B.dom) nmin = std::min(nmin, D.n);
  const int S = (per_blk - 1) / nmin + 2;
  if (form.mean && S > kMaxMeanSlots) {
    set_err(c, "internal: %d component sums per block exceed %d", S, kMaxMeanSlots);
    throw Fail{GNK_ERR_ARG};
  }
  double* mpart = form.mean ? ws<double>(c, "gmmp", (size_t)ncol * nblk * S) : nullptr;
  const unsigned cb = nblocks(ncol, 256);
  k_gmres_init<<<cb, 256, 0, c->stream>>>(ncol, st);
  LAUNCHCHK(c);
  dim3 gv((unsigned)nblk, (unsigned)ncol);
  k_norm_partial<<<gv, kT, 0, c->stream>>>(B.d_dom, B.d_col, b, per_blk, P1, ldp);
  LAUNCHCHK(c);
  k_bnorm<<<(unsigned)ncol, 64, 0, c->stream>>>(P1, nblk, ldp, st);
  LAUNCHCHK(c);

  auto cycle_start = [&](const double* partial) {
    k_cycle_reset<<<1, 1, 0, c->stream>>>(st);
    LAUNCHCHK(c);
    k_cycle_start<<<(unsigned)ncol, 64, 0, c->stream>>>(partial, nblk, ldp, o.tol, st);
    LAUNCHCHK(c);
    // V_0 = r / beta and its pair records for the cycle's first step
    k_stage<<<gv, kT, 0, c->stream>>>(B.d_dom, B.d_col, V, per_blk, form.cw, st, mpart, S);
    LAUNCHCHK(c);
  };
  // r0 = b - A x0 into V_0
  const size_t bytes = sizeof(double) * T;
  if (o.x0) {
    if (o.x0 != x) HIPCHK(c, hipMemcpyAsync(x, o.x0, bytes, hipMemcpyDeviceToDevice, c->stream));
    apply_op(c, B, op, x, V, am);
    k_residual<<<gv, kT, 0, c->stream>>>(B.d_dom, B.d_col, b, V, per_blk, P1, ldp);
  } else {
    HIPCHK(c, hipMemsetAsync(x, 0, bytes, c->stream));
    HIPCHK(c, hipMemcpyAsync(V, b, bytes, hipMemcpyDeviceToDevice, c->stream));
    k_norm_partial<<<gv, kT, 0, c->stream>>>(B.d_dom, B.d_col, V, per_blk, P1, ldp);
  }
  LAUNCHCHK(c);
  cycle_start(P1);

  // host-mapped memory that the last kernel of every Arnoldi step writes: the
  // number of iterating columns and (mixed solves) the residual estimates
  if (!c->pinned) HIPCHK(c, hipHostMalloc((void**)&c->pinned, sizeof(int) * (kMaxRestart + 1), 0));
  if (c->pinned_rel_n < (size_t)ncol * kMaxRestart) {
    if (c->pinned_rel) HIPCHK(c, hipHostFree(c->pinned_rel));
    c->pinned_rel = nullptr;
    HIPCHK(c, hipHostMalloc((void**)&c->pinned_rel, sizeof(double) * ncol * kMaxRestart, 0));
    c->pinned_rel_n = (size_t)ncol * kMaxRestart;
  }
  int* host_live = nullptr;
  double* host_rel = nullptr;
  HIPCHK(c, hipHostGetDevicePointer((void**)&host_live, c->pinned, 0));
  HIPCHK(c, hipHostGetDevicePointer((void**)&host_rel, c->pinned_rel, 0));

  // optional residual history: per column, the true residual at each cycle
  // start followed by the estimate after each of the cycle's Arnoldi steps
  const bool want_hist = o.hist && o.hist_len > 0;
  // With relaxed (mixed) products the residual estimate runs slightly ahead
  // of the true residual, so a mixed cycle aims at half the tolerance; the
  // convergence test itself always uses the FP64 true residual.
  const double stop_tol = mixed ? 0.5 * o.tol : o.tol;
  // One Arnoldi step for every column; the step index l lives on the device
  // (reset at each cycle start, advanced by the last kernel of the step, in
  // st.step for even l and step_odd for odd l), so the same sequence of
  // launches serves every pair of steps and can be captured once.
  auto enqueue_step = [&](bool use_mixed, bool odd) {
    GmresState sl = st;
    if (odd) sl.step = step_odd;
    int* const next = odd ? st.step : step_odd;
    pairs(c, B, P_GM, use_mixed, st.active);
    k_epilogue_dots<<<gv, kT, 0, c->stream>>>(B.d_dom, B.d_col, V, T, form.cout, form.dsel, form.a0, form.dsign,
                                              form.cI, form.cR, mpart, S, st.active, sl.step, per_blk, P1, ldp);
    LAUNCHCHK(c);
    k_gs_update<<<gv, kT, 0, c->stream>>>(B.d_dom, B.d_col, V, T, per_blk, P1, P2, ldp, sl);
    LAUNCHCHK(c);
    k_gs_finish<<<gv, kT, 0, c->stream>>>(B.d_dom, B.d_col, V, T, per_blk, P2, ldp, sl, next, restart, stop_tol,
                                          host_live, host_rel, form.cw, mpart, S);
    LAUNCHCHK(c);
  };
  // Every buffer the step touches exists before a capture (no allocation,
  // upload or event record may happen inside it). Profiling times each pair
  // launch with events and so runs the steps without a graph.
  build_items(c, B, P_GM);
  if (mixed) build_items(c, B, P_GM_MIXED);
  const bool use_graph = c->graphs && !c->prof;
  bool fresh[6] = {};   // cached graph matches this solve's step
  // k (1, 2 or 4) consecutive Arnoldi steps in one launch: the step index
  // lives on the device, and inside a graph the kernels follow each other with
  // no gap, while each graph launch costs a gap of about 13 us
  // profiling: the pair records of each step of the cycle, so that those of the
  // fully masked speculative steps can be left out of the totals
  std::vector<std::pair<size_t, size_t>> step_recs;
  // steps of the launch that starts at step l (even): four while four remain
  // in the cycle, then two, then one
  auto steps_per_launch = [&](int l) { return l + 4 <= restart ? 4 : (l + 2 <= restart ? 2 : 1); };
  // Every argument of the step's launches (enqueue_step and, through pairs,
  // the pair kernels' work lists, shape and variant): the kernels read the
  // domains, columns, work items and vectors through these pointers when they
  // run, so a cached graph whose signature matches needs no new capture. The
  // treecode's launches are not listed: with it the graph is always captured.
  auto step_signature = [&](bool use_mixed, int k) {
    std::vector<uint64_t> sg;
    auto u = [&](uint64_t v) { sg.push_back(v); };
    auto pt = [&](const void* q) { u((uint64_t)(uintptr_t)q); };
    auto fp = [&](double v) { uint64_t b; memcpy(&b, &v, 8); u(b); };
    u((uint64_t)use_mixed); u((uint64_t)k);
    const Batch::ItemSet& IS = B.sets[use_mixed ? P_GM_MIXED : P_GM];
    for (int q = 0; q < 4; ++q) { pt(IS.d[q]); u((uint64_t)IS.cnt[q]); }
    u((uint64_t)B.shape.tpt); pt(B.d_dom); pt(B.d_col); u((uint64_t)B.ndom); u((uint64_t)B.maxN);
    u((uint64_t)(B.dom[0].tz != nullptr));
    u((uint64_t)records32_threads(B, use_mixed ? P_GM_MIXED : P_GM));
    for (const void* q : {(const void*)st.bnorm, (const void*)st.true_relres, (const void*)st.relres,
                          (const void*)st.invbeta, (const void*)st.H, (const void*)st.cs, (const void*)st.sn,
                          (const void*)st.g, (const void*)st.y, (const void*)st.active, (const void*)st.converged,
                          (const void*)st.kdim, (const void*)st.inner_it, (const void*)st.live, (const void*)st.step,
                          (const void*)st.done})
      pt(q);
    u((uint64_t)st.ldh); u((uint64_t)st.hstride);
    pt(V); u((uint64_t)T); u((uint64_t)per_blk); u((uint64_t)nblk); u((uint64_t)ncol); pt(P1); pt(P2);
    u((uint64_t)ldp); pt(step_odd); u((uint64_t)restart); fp(stop_tol); pt(host_live);
    pt(host_rel);
    u((uint64_t)form.cw); u((uint64_t)form.cout); u((uint64_t)form.dsel); fp(form.a0); fp(form.dsign); fp(form.cI);
    fp(form.cR); pt(mpart); u((uint64_t)S); pt(c->stream);
    return sg;
  };
  // capture (or update the cached executable of) the graph of k steps
  auto prepare_step = [&](bool use_mixed, int k) {
    const int m = (use_mixed ? 1 : 0) + (k == 4 ? 4 : 2 * (k - 1));
    hipGraphExec_t& ge = c->step_exec[m];
    if (!fresh[m]) {
      std::vector<uint64_t> sig;
      if (!B.tree.on) sig = step_signature(use_mixed, k);
      if (ge && !sig.empty() && c->step_sig[m] == sig) {
        fresh[m] = true;
        return ge;
      }
      c->step_sig[m].clear();
      hipGraph_t graph = nullptr;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
      try {
        for (int i = 0; i < k; ++i) enqueue_step(use_mixed, (i & 1) != 0);
      } catch (...) {
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(c->stream, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        throw;
      }
      HIPCHK(c, hipStreamEndCapture(c->stream, &graph));
      bool updated = false;
      if (ge) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        updated = hipGraphExecUpdate(ge, graph, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!updated) {
          (void)hipGetLastError();
          (void)hipGraphExecDestroy(ge);
          ge = nullptr;
        }
      }
      hipError_t e = hipSuccess;
      if (!updated) e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) ge = nullptr;
      HIPCHK(c, e);
      c->step_sig[m] = std::move(sig);
      fresh[m] = true;
    }
    return ge;
  };
  auto launch_step = [&](bool use_mixed, int k) {
    if (!use_graph) {
      for (int i = 0; i < k; ++i) {
        const size_t r0 = c->prof_pending.size();
        enqueue_step(use_mixed, (i & 1) != 0);
        step_recs.emplace_back(r0, c->prof_pending.size());
      }
      return;
    }
    HIPCHK(c, hipGraphLaunch(prepare_step(use_mixed, k), c->stream));
  };
  // The first launch's graph is prepared before the host first waits on the
  // stream, so that the capture overlaps the kernels still queued (right-hand
  // side, initial residual) instead of leaving the GPU idle at the cycle
  // start. A mixed solve from a zero start takes mixed steps at once when
  // inner_tol >= 1 (its starting relative residual is 1); a wrong guess only
  // costs a capture.
  if (use_graph) (void)prepare_step(mixed && !o.x0 && o.inner_tol >= 1.0, steps_per_launch(0));

  std::vector<int> outer(ncol, 0), conv(ncol, 0), mixed_steps(ncol, 0), refine(ncol, 0);
  std::vector<int> hist_cnt(ncol, 0), prev_inner(ncol, 0);
  bool sums_of_x = false;
  bool mixed_now = false;
  bool refine_capped = false;   // max_refine cycles with mixed products done: FP64 from here on
  int mixed_cycles = 0;
  while ((int)c->step_ev.size() < kMaxRestart) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->step_ev.push_back(e);
  }
  // per-column results read back through host-mapped memory at each cycle
  // start: [live, converged.., inner_it..] and [true_relres.., relres..]
  char* hio = hostio(c, (sizeof(int) * 2 + sizeof(double) * 2) * (ncol + 1));
  int* hi = reinterpret_cast<int*>(hio);
  double* hd = reinterpret_cast<double*>(hio + sizeof(int) * 2 * (ncol + 1));
  int* hi_dev = hostio_dev(c, hi);
  double* hd_dev = hostio_dev(c, hd);
  bool published = false;   // the host copy holds the final state
  // after each publish: the history entries of the cycle that just ended (its
  // steps' estimates, then the true residual that starts the next cycle)
  auto record_hist = [&](bool first) {
    if (!want_hist) return;
    for (int q = 0; q < ncol; ++q) {
      const int inner_q = hi[1 + ncol + q];
      const int steps = inner_q - prev_inner[q];
      if (!first && steps <= 0) continue;
      double* hq = o.hist + (size_t)q * o.hist_len;
      for (int t = 0; t < steps && hist_cnt[q] < o.hist_len; ++t) hq[hist_cnt[q]++] = c->pinned_rel[(size_t)t * ncol + q];
      if (hist_cnt[q] < o.hist_len) hq[hist_cnt[q]++] = hd[q];
      prev_inner[q] = inner_q;
    }
  };
  // From a zero start the first cycle's residual is b itself, so every column
  // with b != 0 iterates and the host need not wait for the cycle-start state
  // (a column with b = 0 takes no Arnoldi step, and its outer count is set
  // back at the end). Mixed solves and residual histories read that state.
  const bool lazy_start = !o.x0 && !mixed && !want_hist;
  for (int cyc = 0; cyc < o.maxit; ++cyc) {
    if (cyc > 0 || !lazy_start) {
      k_publish_cycle<<<nblocks(ncol + 1), kT, 0, c->stream>>>(st, ncol, hi_dev, hd_dev);
      LAUNCHCHK(c);
      HIPCHK(c, hipStreamSynchronize(c->stream));
      record_hist(cyc == 0);
      const int live = hi[0];
      for (int q = 0; q < ncol; ++q) conv[q] = hi[1 + q];
      if (live == 0) {
        published = true;
        break;
      }
    }
    // a cycle whose starting (FP64) residual is already below inner_tol
    // takes mixed products from its first step
    if (mixed && !mixed_now && !refine_capped) {
      double mx = 0.0;
      for (int q = 0; q < ncol; ++q)
        if (!conv[q]) mx = std::max(mx, hd[q]);
      if (mx <= o.inner_tol) mixed_now = true;
    }
    for (int q = 0; q < ncol; ++q)
      if (!conv[q]) outer[q] += 1;
    // Arnoldi steps, up to four per launch. The host looks one launch behind
    // the device: before enqueuing the next launch it waits for the last step
    // of the one before the current and reads how many columns are still
    // iterating, so the queue never drains and at most seven speculative steps
    // run (fully masked) after the last column stops.
    step_recs.clear();
    bool cycle_mixed = false;
    // The host also tracks the largest residual estimate of the steps it
    // reads: when the estimates' geometric rate over its last two readings
    // says that the launch just enqueued ends the cycle (every column at the
    // stop tolerance), it waits for that launch instead of enqueuing another
    // one of fully masked steps; a wrong guess costs a round trip.
    double seen_rel = -1.0;
    int seen_step = -1;
    // (l is even at every launch: its steps are the even-odd pairs of enqueue_step)
    for (int l = 0; l < restart;) {
      const bool use_mixed = mixed && mixed_now;
      cycle_mixed = cycle_mixed || use_mixed;
      const int k = steps_per_launch(l);
      if (use_mixed)
        for (int q = 0; q < ncol; ++q)
          if (!conv[q]) mixed_steps[q] += k;
      launch_step(use_mixed, k);
      HIPCHK(c, hipEventRecord(c->step_ev[l + k - 1], c->stream));
      const int prev = l - 1;   // last step of the previous launch
      l += k;
      if (prev >= 0) {
        HIPCHK(c, hipEventSynchronize(c->step_ev[prev]));
        if (c->pinned[prev] == 0) break;
        double mx = 0.0;
        for (int q = 0; q < ncol; ++q) mx = std::max(mx, c->pinned_rel[(size_t)prev * ncol + q]);
        if (mixed && !mixed_now && !refine_capped && mx <= o.inner_tol) mixed_now = true;
        if (seen_step >= 0 && mx > stop_tol && mx < seen_rel && l < restart) {
          const double rate = std::log(mx / seen_rel) / (double)(prev - seen_step);   // per step, < 0
          const double need = std::log(stop_tol / mx) / rate;                       // steps after prev
          if (need <= (double)(l - 1 - prev)) {
            HIPCHK(c, hipEventSynchronize(c->step_ev[l - 1]));
            if (c->pinned[l - 1] == 0) break;
          }
        }
        seen_rel = mx;
        seen_step = prev;
      }
    }
    if (c->prof && !step_recs.empty()) {
      // steps after the first one that left no column iterating did no work
      HIPCHK(c, hipStreamSynchronize(c->stream));
      int dead = -1;
      for (int t = 0; t < (int)step_recs.size() && dead < 0; ++t)
        if (c->pinned[t] == 0) dead = t;
      if (dead >= 0)
        for (int t = dead + 1; t < (int)step_recs.size(); ++t)
          for (size_t r = step_recs[t].first; r < step_recs[t].second; ++r) c->prof_pending[r].spec = true;
    }
    k_backsolve<<<(unsigned)ncol, 64, 0, c->stream>>>(st);
    LAUNCHCHK(c);
    k_xupdate<<<col_grid(B), kT, 0, c->stream>>>(B.d_dom, B.d_col, V, T, x, st);
    LAUNCHCHK(c);
    // true residual of the new iterate (FP64 product) and the next cycle's start
    apply_op(c, B, op, x, V, am);
    sums_of_x = (op == GNK_OP_FB || op == GNK_OP_FB_U);
    k_residual<<<gv, kT, 0, c->stream>>>(B.d_dom, B.d_col, b, V, per_blk, P1, ldp);
    LAUNCHCHK(c);
    cycle_start(P1);
    // a cycle with mixed products followed by this FP64 residual is one step of
    // iterative refinement; after max_refine of them the cycles stay FP64
    if (cycle_mixed) {
      for (int q = 0; q < ncol; ++q)
        if (!conv[q]) refine[q] += 1;
      if (o.max_refine > 0 && ++mixed_cycles >= o.max_refine) {
        refine_capped = true;
        mixed_now = false;
      }
    }
    if (c->log) {
      std::vector<double> tr(ncol);
      HIPCHK(c, hipMemcpyAsync(tr.data(), st.true_relres, sizeof(double) * ncol, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      double mx = 0;
      for (double v : tr) mx = std::max(mx, v);
      fprintf(stderr, "[gnk] op %d cycle %d max true relres %.3e%s\n", op, cyc + 1, mx,
              mixed_now ? " (mixed products)" : "");
    }
  }
  GmresOut out;
  out.sums_of_x = sums_of_x;
  out.info.resize(ncol);
  std::vector<double> rel(ncol), trel(ncol);
  std::vector<int> inner(ncol);
  if (!published) {   // maxit cycles ran: publish the state after the last cycle start
    k_publish_cycle<<<nblocks(ncol + 1), kT, 0, c->stream>>>(st, ncol, hi_dev, hd_dev);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    record_hist(false);
  }
  for (int q = 0; q < ncol; ++q) {
    conv[q] = hi[1 + q];
    inner[q] = hi[1 + ncol + q];
    trel[q] = hd[q];
    rel[q] = hd[ncol + q];
    if (lazy_start && inner[q] == 0) outer[q] = 0;
  }
  out.all_converged = true;
  for (int q = 0; q < ncol; ++q) {
    gnk_info& I = out.info[q];
    I.flag = conv[q] ? 0 : 1;
    I.outer_it = outer[q];
    I.inner_it = inner[q];
    I.mixed_steps = std::min(mixed_steps[q], I.inner_it);   // the host count includes speculative steps
    I.relres = rel[q];
    I.true_relres = trel[q];
    I.refine_steps = refine[q];
    I.hist_count = hist_cnt[q];
    if (!conv[q]) out.all_converged = false;
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
  r.x0 = nullptr;
  if (o) r = *o;
  if (r.restart < 1 || r.restart > kMaxRestart || r.maxit < 1 || !(r.tol > 0.0) || r.tol >= 1.0 ||
      (r.prec != GNK_FP64 && r.prec != GNK_MIXED) || (r.no_subtraction != 0 && r.no_subtraction != 1) ||
      r.max_refine < 0 || r.hist_len < 0 || (r.hist_len > 0 && !r.hist) ||
      !(r.far_tol >= 0.0) || (r.far_tol > 0.0 && (r.far_tol < 1e-15 || r.far_tol > 0.1 || r.prec != GNK_FP64))) {
    set_err(c, "bad options: restart %d (1..%d), maxit %d (>=1), tol %g (0..1), prec %d, no_subtraction %d, "
            "far_tol %g (0, or 1e-15..0.1 with GNK_FP64), max_refine %d (>=0), hist_len %d (>=0, hist set "
            "when > 0)", r.restart, kMaxRestart, r.maxit, r.tol, r.prec, r.no_subtraction, r.far_tol,
            r.max_refine, r.hist_len);
    throw Fail{GNK_ERR_ARG};
  }
  // mixed products once the residual estimate is below 5e6 tol, but not
  // before 1e-4: the products' relative error (about 1e-8) then adds at most
  // about tol/2 to the final residual over the remaining steps, so the mixed
  // cycle ends below tol without a restart (measured on the close-boundary
  // workload: switching at 1e8 tol left a true residual of about 3 tol at the
  // end of the cycle, and the restart that followed cost about 45 extra steps)
  if (r.inner_tol <= 0) r.inner_tol = std::min(1e-4, r.tol * 5e6);
  return r;
}

// ------------------------------------------------------------- autotuner
// Picks the pair-kernel launch shape (targets per lane, sources per
// workgroup) for a batch by timing the Cauchy sums of one product per
// candidate; results are cached per batch signature in the context and, with
// GNK_TUNE_CACHE=path, in a text file ("key tpt chunk" per line).
std::string tune_key(const gnk_ctx* c, int ndom, const gnk_domain* doms, const int* ncols, bool mixed) {
  std::vector<std::pair<int64_t, int>> v;
  for (int d = 0; d < ndom; ++d) v.push_back({doms[d].m1 * doms[d].n, ncols[d]});
  std::sort(v.begin(), v.end());
  uint64_t h = 1469598103934665603ull;   // FNV-1a over the sorted (N, ncols) list
  for (auto& p : v) {
    h = (h ^ (uint64_t)p.first) * 1099511628211ull;
    h = (h ^ (uint64_t)p.second) * 1099511628211ull;
  }
  std::ostringstream k;
  k << "cu" << c->num_cu << (mixed ? "m" : "d") << "_" << v.size() << "_" << std::hex << h;
  return k.str();
}

void load_tune_cache(gnk_ctx* c) {
  if (c->tune_loaded) return;
  c->tune_loaded = true;
  const char* path = getenv("GNK_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string key, rest;
  while (f >> key && std::getline(f, rest)) c->tune[key] = rest;
}

void store_tune_cache(gnk_ctx* c, const std::string& key, const std::string& val) {
  c->tune[key] = val;
  if (const char* path = getenv("GNK_TUNE_CACHE")) {
    std::ofstream f(path, std::ios::app);
    f << key << " " << val << "\n";
  }
}

PairShape tuned_shape(gnk_ctx* c, int ndom, const gnk_domain* doms, const int* ncols, bool mixed,
                      const double* x_flat, const std::vector<int64_t>& col_off, int64_t T) {
  PairShape def;
  def.tpt = 1;
  def.chunk = 2048;
  const char* env = getenv("GNK_TUNE");
  if (env && atoi(env) == 0) return def;
  load_tune_cache(c);
  const std::string key = tune_key(c, ndom, doms, ncols, mixed);
  auto it = c->tune.find(key);
  if (it != c->tune.end()) {
    std::istringstream s(it->second);
    PairShape p;
    if (s >> p.tpt >> p.chunk) return p;
  }
  const std::vector<PairShape> cand = {{1, 512}, {1, 2048}, {2, 1024}, {2, 4096}};
  hipEvent_t a, b;
  HIPCHK(c, hipEventCreate(&a));
  HIPCHK(c, hipEventCreate(&b));
  double best = 1e300;
  PairShape bestp = def;
  const bool prof = c->prof;
  c->prof = false;
  for (const PairShape& p : cand) {
    Batch B;
    build_batch(c, B, ndom, doms, ncols, col_off, T, false, mixed, p);
    k_rho<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom);
    LAUNCHCHK(c);
    k_weights<<<dim3((unsigned)B.maxm1, (unsigned)B.ncol), kT, 0, c->stream>>>(
        B.d_dom, B.d_col, C_RHO, x_flat, nullptr, 0, nullptr, B.maxm1);
    LAUNCHCHK(c);
    build_items(c, B, P_GM);
    if (&p == &cand[0]) pairs(c, B, P_GM, mixed, nullptr);   // first launch of the kernels
    HIPCHK(c, hipEventRecord(a, c->stream));
    pairs(c, B, P_GM, mixed, nullptr);
    HIPCHK(c, hipEventRecord(b, c->stream));
    HIPCHK(c, hipEventSynchronize(b));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, a, b));
    if (c->log) fprintf(stderr, "[gnk] tune tpt %d chunk %d: %.3f ms\n", p.tpt, p.chunk, ms);
    if (ms < best) {
      best = ms;
      bestp = p;
    }
  }
  c->prof = prof;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::ostringstream v;
  v << bestp.tpt << " " << bestp.chunk;
  store_tune_cache(c, key, v.str());
  return bestp;
}

// ----------------------------------------------------------- FBIE / FBIEad
// gam, mu, h: flat vectors of the batch (h may be null).
GmresOut fbie_batch(gnk_ctx* c, Batch& B, const double* gam, const gnk_opts& o, double* mu, double* h) {
  const int64_t T = B.T;
  validate_enqueue(c, B, gam, T);
  k_rho<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom);
  LAUNCHCHK(c);
  // one launch for E(rho) (leading column) and E(rho gamma) (data columns)
  k_weights<<<dim3((unsigned)B.maxm1, (unsigned)B.ncol), kT, 0, c->stream>>>(
      B.d_dom, B.d_col, C_RHO, gam, nullptr, 1, nullptr, B.maxm1);
  LAUNCHCHK(c);
  pairs(c, B, P_SETUP, false, nullptr);
  k_diag_fbie<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom, 1, 1);
  LAUNCHCHK(c);
  // b = -y = -(D - diag(D1) + Lhat) gamma
  double* b = ws<double>(c, "rhs", T);
  k_epilogue<<<col_grid(B), kT, 0, c->stream>>>(B.d_dom, B.d_col, gam, C_A, D_D, 0.0, 1.0, 0.0, 1.0, nullptr, 0,
                                                nullptr, 1, b);
  LAUNCHCHK(c);
  circulant(c, B, gam, b, -1.0);
  // f_B(gamma) from the same sums, for h; without singularity subtraction the
  // operator is I - B - diag(Nd) (Nd the diagonal limit (e:N-tt))
  const bool unsub = o.no_subtraction != 0;
  if (unsub) setup_ndiag(c, B);
  double* fbg = nullptr;
  if (h) {
    fbg = ws<double>(c, "fbg", T);
    if (unsub)
      k_epilogue<<<col_grid(B), kT, 0, c->stream>>>(B.d_dom, B.d_col, gam, C_A, D_BU, 1.0, -1.0, 1.0, 0.0, nullptr,
                                                    0, nullptr, 1, fbg);
    else
      k_epilogue<<<col_grid(B), kT, 0, c->stream>>>(B.d_dom, B.d_col, gam, C_A, D_B, 2.0, 1.0, 1.0, 0.0, nullptr, 0,
                                                    nullptr, 1, fbg);
    LAUNCHCHK(c);
  }
  validate_finish(c);
  // (2I + diag(B1) - B) mu = b, or (I - B - diag(Nd)) mu = b
  GmresOut g = gmres(c, B, unsub ? GNK_OP_FB_U : GNK_OP_FB, b, o, mu, o.prec == GNK_MIXED);
  if (h) {
    // h = [(D - diag(D1) + Lhat) mu - (2I + diag(B1) - B) gamma] / 2; D mu from
    // the sums of GMRES's last (FP64) residual product of mu when it left them
    ApplyArgs ah;
    ah.reuse_sums = g.sums_of_x;
    apply_op(c, B, GNK_OP_FC, mu, h, ah);
    k_axpby<<<nblocks(T), kT, 0, c->stream>>>(-0.5, fbg, 0.5, h, T);
    LAUNCHCHK(c);
  }
  return g;
}

GmresOut fbiead_batch(gnk_ctx* c, Batch& B, const double* gam, const gnk_opts& o, double* mu) {
  validate_enqueue(c, B, gam, B.T);
  k_rho<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom);
  LAUNCHCHK(c);
  setup_evec(c, B);
  validate_finish(c);
  if (o.no_subtraction) {
    setup_ndiag(c, B);
    return gmres(c, B, GNK_OP_GB_U, gam, o, mu, o.prec == GNK_MIXED);
  }
  return gmres(c, B, GNK_OP_GB, gam, o, mu, o.prec == GNK_MIXED);
}

template <class F>
gnk_status guarded(gnk_ctx* c, F&& f) {
  if (!c) return GNK_ERR_ARG;
  c->err.clear();
  try {
    HIPCHK(c, hipSetDevice(c->device));
    // uploads of the previous call have completed (every call ends synchronised)
    c->host_keep.clear();
    return f();
  } catch (const Fail& e) {
    (void)hipStreamSynchronize(c->stream);
    return e.st;
  } catch (const std::bad_alloc&) {
    set_err(c, "host allocation failed");
    (void)hipStreamSynchronize(c->stream);
    return GNK_ERR_OOM;
  }
}

// Batch of one domain whose flat vectors are the caller's N x nrhs arrays.
void single_batch(gnk_ctx* c, Batch& B, const gnk_domain* d, int nrhs, bool adjoint, bool mixed,
                  bool second = false) {
  check_domain(c, d, adjoint, second);
  std::vector<int64_t> off{0};
  build_batch(c, B, 1, d, &nrhs, off, d->m1 * d->n * (int64_t)nrhs, adjoint, mixed, PairShape{});
  B.second = second || adjoint;
}


// ------------------------------------------------------- differentiation
// Adjoint of FBIE (transpose of eq. (e:sys)):
//   lam = Aop^{-T} (Cop^T g_h / 2 + g_mu),   g_gam = -Aop^T g_h / 2 - Cop^T lam.
GmresOut fbie_adjoint_batch(gnk_ctx* c, Batch& B, const double* g_mu, const double* g_h, const gnk_opts& o,
                            double* lam, double* g_gam) {
  const int64_t T = B.T;
  if (g_mu) validate(c, B, g_mu, T);
  if (g_h) validate(c, B, g_h, T);
  k_rho<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom);
  LAUNCHCHK(c);
  setup_diag(c, B);
  double* b = ws<double>(c, "adj_rhs", T);
  if (g_h) {
    apply_op(c, B, GNK_OP_FC_T, g_h, b);
    if (g_mu) k_axpby<<<nblocks(T), kT, 0, c->stream>>>(1.0, g_mu, 0.5, b, T);
    else k_axpby<<<nblocks(T), kT, 0, c->stream>>>(0.0, b, 0.5, b, T);
    LAUNCHCHK(c);
  } else {
    HIPCHK(c, hipMemcpyAsync(b, g_mu, sizeof(double) * T, hipMemcpyDeviceToDevice, c->stream));
  }
  GmresOut g = gmres(c, B, GNK_OP_FB_T, b, o, lam, o.prec == GNK_MIXED);
  if (g_gam) {
    apply_op(c, B, GNK_OP_FC_T, lam, g_gam);
    if (g_h) {
      double* t = ws<double>(c, "adj_tmp", T);
      apply_op(c, B, GNK_OP_FB_T, g_h, t);
      k_axpby<<<nblocks(T), kT, 0, c->stream>>>(-0.5, t, -1.0, g_gam, T);
    } else {
      k_axpby<<<nblocks(T), kT, 0, c->stream>>>(0.0, g_gam, -1.0, g_gam, T);
    }
    LAUNCHCHK(c);
  }
  return g;
}

// Gradient of s = sum_t coef_t u_t^T Op_t v_t with respect to eta, eta', A:
// weights per source, first- and second-order Cauchy sums, per-node epilogue.
void geom_vjp(gnk_ctx* c, const gnk_domain* d, int nterms, const int* ops, const double* coef,
              const double* const* u, const double* const* v, double2* g_eta, double2* g_etap, double2* g_A) {
  Batch B;
  single_batch(c, B, d, 1, false, false);
  const int N = B.dom[0].N;
  {
    // finiteness of the domain data and of every term vector
    int* flags = ws<int>(c, "flags", 1);
    HIPCHK(c, hipMemsetAsync(flags, 0, sizeof(int), c->stream));
    k_validate<<<node_grid(B), kT, 0, c->stream>>>(B.d_dom, 0, flags);
    LAUNCHCHK(c);
    for (int t = 0; t < nterms; ++t) {
      k_check_finite<<<nblocks(N), kT, 0, c->stream>>>(u[t], N, flags);
      k_check_finite<<<nblocks(N), kT, 0, c->stream>>>(v[t], N, flags);
    }
    LAUNCHCHK(c);
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
  }
  // group the terms by their v vector
  std::vector<const double*> gv;
  std::vector<std::vector<int>> members;
  for (int t = 0; t < nterms; ++t) {
    size_t g = 0;
    while (g < gv.size() && gv[g] != v[t]) ++g;
    if (g == gv.size()) {
      gv.push_back(v[t]);
      members.emplace_back();
    }
    members[g].push_back(t);
  }
  std::vector<GeomTerm> terms;
  std::vector<GeomGroup> groups;
  for (size_t g = 0; g < gv.size(); ++g) {
    const int t0 = (int)terms.size();
    for (int t : members[g]) {
      const double cf = coef ? coef[t] : 1.0;
      terms.push_back(GeomTerm{u[t], ops[t] == GNK_OP_FB ? make_double2(0.0, cf) : make_double2(cf, 0.0)});
    }
    groups.push_back(GeomGroup{gv[g], t0, (int)terms.size()});
  }
  const int G = (int)groups.size();
  const int nw = 2 * G + 2;
  // enough workgroups for two rounds of the wave slots, at least 256 sources each
  const int64_t tiles = (N + 63) / 64;
  int64_t splits = (2 * slots_of(c) + 4 * tiles - 1) / (4 * tiles);
  splits = std::max<int64_t>(1, std::min<int64_t>(splits, std::min<int64_t>(64, std::max<int64_t>(1, N / 256))));
  int64_t chunk = (N + splits - 1) / splits;
  chunk = (chunk + 3) / 4 * 4;
  splits = (N + chunk - 1) / chunk;
  const GeomTerm* dterms = upload(c, "g_terms", terms);
  const GeomGroup* dgroups = upload(c, "g_groups", groups);
  double2* rec = ws<double2>(c, "g_rec", (size_t)N * (1 + nw));
  double2* Ut = ws<double2>(c, "g_U", (size_t)G * N);
  double2* P = ws<double2>(c, "g_P", N);
  double2* parts = ws<double2>(c, "g_parts", (size_t)splits * nw * 2 * N);
  const DomDev& D = B.dom[0];
  HIPCHK(c, launch_geom_weights(D.eta, D.etap, D.A, N, dterms, dgroups, G, nw, rec, Ut, P, c->stream));
  HIPCHK(c, launch_cauchy12(rec, nw, N, nw, (int)chunk, (int)splits, parts, c->stream));
  HIPCHK(c, launch_geom_epilogue(D.etap, D.A, N, D.n, dgroups, G, Ut, P, parts, nw, (int)splits, g_eta, g_etap, g_A,
                                 c->stream));
}

std::mutex scratch_mu;
std::map<int, char*> scratch_addr;   // device -> address of its scratch array

// the current device's scratch address (nullptr if the runtime cannot give it)
char* scratch_of_device(int device) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  auto it = scratch_addr.find(device);
  if (it != scratch_addr.end()) return it->second;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  scratch_addr[device] = static_cast<char*>(p);
  return static_cast<char*>(p);
}

// While alive, ws() of this context carves buffers from [base, base + cap).
struct ArenaScope {
  gnk_ctx* c;
  ArenaScope(gnk_ctx* c_, char* base, size_t cap) : c(c_) {
    c->arena = base;
    c->arena_cap = cap;
    c->arena_used = 0;
  }
  ~ArenaScope() {
    c->arena = nullptr;
    c->arena_cap = 0;
    c->arena_used = 0;
  }
};

// S = E w for gnk_cauchy_sum and gnk_cauchy_sum_noalloc
void cauchy_sum(gnk_ctx* c, int64_t N, const void* eta, const void* w, int nrhs, void* S) {
  if (N < 1 || N > ((int64_t)1 << 30) || nrhs < 1 || !eta || !w || !S || w == S) {
    set_err(c, "bad arguments to gnk_cauchy_sum");
    throw Fail{GNK_ERR_ARG};
  }
  // a pseudo-domain of one component holding the N nodes (the even mesh
  // size only passes the domain check; the node count is N)
  gnk_domain d{};
  d.m1 = 1;
  d.n = N + (N & 1);
  d.eta = d.etap = d.A = eta;
  Batch B;
  std::vector<int64_t> off{0};
  build_batch(c, B, 1, &d, &nrhs, off, N * (int64_t)nrhs, false, false, PairShape{}, N);
  k_pack_records<<<nblocks(N), kT, 0, c->stream>>>(B.d_dom, static_cast<const double2*>(w), nrhs);
  LAUNCHCHK(c);
  pairs(c, B, P_GM, false, nullptr);
  k_reduce_parts<<<dim3(nblocks(N), (unsigned)nrhs), kT, 0, c->stream>>>(B.d_dom, static_cast<double2*>(S));
  LAUNCHCHK(c);
  HIPCHK(c, hipStreamSynchronize(c->stream));
}

}  // namespace
}  // namespace gnk

using namespace gnk;

extern "C" {

const char* gnk_version(void) { return "gnk 0.2.0 (gfx950, direct Cauchy sums, batched)"; }

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
  if (const char* s = getenv("GNK_GRAPH")) c->graphs = atoi(s) != 0;
  // a blocking stream of default priority: ordered with the legacy null
  // stream, and capturable (the null stream cannot be captured)
  if (hipStreamCreate(&c->own_stream) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return GNK_ERR_HIP;
  }
  c->stream = c->own_stream;
  c->scratch = scratch_of_device(device);
  *out = c;
  return GNK_OK;
}

gnk_status gnk_destroy(gnk_ctx* c) {
  if (!c) return GNK_ERR_ARG;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& kv : c->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto e : c->step_ev) (void)hipEventDestroy(e);
  for (auto& g : c->step_exec)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto& r : c->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->val_ev) (void)hipEventDestroy(c->val_ev);
  if (c->vflags) (void)hipHostFree(c->vflags);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->pinned_rel) (void)hipHostFree(c->pinned_rel);
  if (c->hostio) (void)hipHostFree(c->hostio);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
  return GNK_OK;
}

gnk_status gnk_set_stream(gnk_ctx* c, void* s) {
  if (!c) return GNK_ERR_ARG;
  c->stream = s ? static_cast<hipStream_t>(s) : c->own_stream;
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
      gnk_prof& A = c->prof_acc;
      c->ev_pool.push_back(r.a);
      c->ev_pool.push_back(r.b);
      if (r.spec) continue;
      if (r.fft) {
        A.launches_fft += 1;
        A.ms_fft += ms;
        A.bytes_fft += r.fft_bytes;
        continue;
      }
      A.launches += 1;
      A.ms += ms;
      A.pair_cols += r.pair_cols;
      A.flops += r.flops;
      if (r.tree) {
        A.launches_tree += 1;
        A.ms_tree += ms;
        A.flops_tree += r.tree_flops;
      }
      if (r.mixed) {
        A.launches_mixed += 1;
        A.ms_mixed += ms;
        A.pair_cols_mixed += r.pair_cols;
      } else if (r.single) {
        A.launches1 += 1;
        A.ms1 += ms;
        A.pairs1 += r.pairs1;
      }
    }
    c->prof_pending.clear();
    if (out) *out = c->prof_acc;
    if (reset) c->prof_acc = gnk_prof{};
    return GNK_OK;
  });
}

gnk_status gnk_cauchy_sum(gnk_ctx* c, int64_t N, const void* eta, const void* w, int nrhs, void* S) {
  return guarded(c, [&]() -> gnk_status {
    cauchy_sum(c, N, eta, w, nrhs, S);
    return GNK_OK;
  });
}

gnk_status gnk_cauchy_sum_noalloc(gnk_ctx* c, int64_t N, const void* eta, const void* w, int nrhs, void* S) {
  return guarded(c, [&]() -> gnk_status {
    if (!c->scratch) {
      set_err(c, "gnk_cauchy_sum_noalloc: the scratch array's address on device %d is unknown", c->device);
      throw Fail{GNK_ERR_HIP};
    }
    ArenaScope scope(c, c->scratch, kScratchBytes);
    cauchy_sum(c, N, eta, w, nrhs, S);
    return GNK_OK;
  });
}


// Boundary values of the map onto the unit disc (bounded G) or the extended plane
// (unbounded G) with slits, from one FBIE solve (theta == NULL: pi/2 on every
// component). level[k] = hbar_k - hbar_0 sin(theta_k) (bounded), hbar_k (unbounded).
static gnk_status slit_map(gnk_ctx* c, const char* name, int64_t m1, int64_t n, const void* eta, const void* etap,
                           int bounded, const double* alpha, const double* theta, const gnk_opts* opts, void* f,
                           double* level, gnk_info* info) {
  if (!eta || !etap || !alpha || !f || f == eta || f == etap || m1 < 1 || n < 2 || (bounded != 0 && bounded != 1) ||
      !std::isfinite(alpha[0]) || !std::isfinite(alpha[1])) {
    set_err(c, "bad arguments to %s", name);
    throw Fail{GNK_ERR_ARG};
  }
  gnk_opts o = resolve_opts(c, opts);
  if (o.no_subtraction) {
    set_err(c, "the map takes the paper's method (no_subtraction = 0)");
    throw Fail{GNK_ERR_ARG};
  }
  const int64_t N = m1 * n;
  if (N > ((int64_t)1 << 30)) {
    set_err(c, "N = (m+1) n = %lld exceeds 2^30", (long long)N);
    throw Fail{GNK_ERR_ARG};
  }
  // rot_k = exp(i (pi/2 - theta_k)) = (sin theta_k, cos theta_k)
  std::vector<double2> rot((size_t)m1, make_double2(1.0, 0.0));
  if (theta) {
    if (bounded && std::fabs(theta[0] - 0.5 * M_PI) > 1e-12) {
      set_err(c, "theta_0 must be pi/2 (the outer boundary maps onto the unit circle)");
      throw Fail{GNK_ERR_ARG};
    }
    for (int64_t k = bounded; k < m1; ++k) {
      if (!std::isfinite(theta[k])) {
        set_err(c, "theta[%lld] is not finite", (long long)k);
        throw Fail{GNK_ERR_ARG};
      }
      rot[k] = make_double2(std::cos(0.5 * M_PI - theta[k]), std::sin(0.5 * M_PI - theta[k]));
    }
  }
  double2* A = ws<double2>(c, "s_A", N);
  double* gam = ws<double>(c, "s_gam", N);
  double* mu = ws<double>(c, "s_mu", N);
  double* h = ws<double>(c, "s_h", N);
  double* hbar = ws<double>(c, "s_hbar", m1);
  double* wind = ws<double>(c, "s_wind", m1);
  double2* rot_d = ws<double2>(c, "s_rot", m1);
  HIPCHK(c, hipMemcpyAsync(rot_d, rot.data(), sizeof(double2) * m1, hipMemcpyHostToDevice, c->stream));
  k_slit_setup<<<(unsigned)m1, kT, 0, c->stream>>>(static_cast<const double2*>(eta), (int)n, bounded, alpha[0],
                                                    alpha[1], rot_d, A, gam, wind);
  LAUNCHCHK(c);
  std::vector<double> w((size_t)m1);
  HIPCHK(c, hipMemcpyAsync(w.data(), wind, sizeof(double) * m1, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int64_t k = 0; k < m1; ++k) {
    const int want = (k == 0 && bounded) ? 1 : 0;
    if (!(std::fabs(w[k] - 2.0 * M_PI * want) < 1.0)) {
      set_err(c, "alpha is not in G: the boundary component %lld winds %.3g times around it (expected %d)",
              (long long)k, w[k] / (2.0 * M_PI), want);
      throw Fail{GNK_ERR_ARG};
    }
  }
  gnk_domain d{};
  d.m1 = m1;
  d.n = n;
  d.eta = eta;
  d.etap = etap;
  d.A = A;
  Batch B;
  single_batch(c, B, &d, 1, false, o.prec == GNK_MIXED);
  if (o.far_tol > 0.0) build_tree(c, B, o.far_tol);
  GmresOut g = fbie_batch(c, B, gam, o, mu, h);
  k_comp_means<<<(unsigned)m1, kT, 0, c->stream>>>(h, (int)n, hbar);
  LAUNCHCHK(c);
  k_slit_map<<<nblocks(N), kT, 0, c->stream>>>(static_cast<const double2*>(eta), bounded, alpha[0], alpha[1], rot_d,
                                               gam, mu, hbar, N, (int)n, static_cast<double2*>(f));
  LAUNCHCHK(c);
  std::vector<double> hb((size_t)m1);
  HIPCHK(c, hipMemcpyAsync(hb.data(), hbar, sizeof(double) * m1, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (level)
    for (int64_t k = 0; k < m1; ++k) level[k] = bounded ? hb[k] - hb[0] * rot[k].x : hb[k];
  if (info) info[0] = g.info[0];
  return g.all_converged ? GNK_OK : GNK_NOT_CONVERGED;
}

gnk_status gnk_circular_slit_map(gnk_ctx* c, int64_t m1, int64_t n, const void* eta, const void* etap,
                                 const double* alpha, const gnk_opts* opts, void* f, double* radii, gnk_info* info) {
  return guarded(c, [&]() -> gnk_status {
    std::vector<double> level((size_t)std::max<int64_t>(m1, 1));
    const gnk_status st =
        slit_map(c, "gnk_circular_slit_map", m1, n, eta, etap, 1, alpha, nullptr, opts, f, level.data(), info);
    if (radii)
      for (int64_t k = 0; k < m1; ++k) radii[k] = std::exp(level[k]);
    return st;
  });
}

gnk_status gnk_slit_map(gnk_ctx* c, int64_t m1, int64_t n, const void* eta, const void* etap, int bounded,
                        const double* alpha, const double* theta, const gnk_opts* opts, void* f, double* level,
                        gnk_info* info) {
  return guarded(c, [&]() -> gnk_status {
    return slit_map(c, "gnk_slit_map", m1, n, eta, etap, bounded, alpha, theta, opts, f, level, info);
  });
}

gnk_status gnk_cauchy_sum_tree(gnk_ctx* c, int64_t N, const void* eta, const void* w, int nrhs, double far_tol,
                               void* S) {
  return guarded(c, [&]() -> gnk_status {
    if (N < 1 || N > ((int64_t)1 << 30) || nrhs < 1 || !eta || !w || !S || w == S || !(far_tol >= 1e-15) ||
        far_tol > 0.1) {
      set_err(c, "bad arguments to gnk_cauchy_sum_tree");
      throw Fail{GNK_ERR_ARG};
    }
    gnk_domain d{};
    d.m1 = 1;
    d.n = N + (N & 1);
    d.eta = d.etap = d.A = eta;
    Batch B;
    std::vector<int64_t> off{0};
    build_batch(c, B, 1, &d, &nrhs, off, N * (int64_t)nrhs, false, false, PairShape{}, N);
    build_tree(c, B, far_tol);
    k_pack_records<<<nblocks(N), kT, 0, c->stream>>>(B.d_dom, static_cast<const double2*>(w), nrhs);
    LAUNCHCHK(c);
    pairs(c, B, P_GM, false, nullptr);
    k_reduce_parts<<<dim3(nblocks(N), (unsigned)nrhs), kT, 0, c->stream>>>(B.d_dom, static_cast<double2*>(S));
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GNK_OK;
  });
}

// The Cauchy integral at interior points; far_tol > 0: the sums by the treecode
// (the node tree as for gnk_cauchy_sum_tree, target tiles of the points)
static gnk_status fcau(gnk_ctx* c, const char* name, int64_t m1, int64_t n, const void* eta, const void* etap,
                       const void* f, int nrhs, const void* z, int64_t nz, const void* finf, double far_tol,
                       void* fz) {
  {
    const int64_t N = m1 * n;
    if (m1 < 1 || n < 1 || N > ((int64_t)1 << 30) || nz < 1 || nz > ((int64_t)1 << 30) || nrhs < 1 ||
        nrhs > 4096 || !eta || !etap || !f || !z || !fz || fz == f || fz == z || fz == eta || fz == etap ||
        (far_tol != 0.0 && !(far_tol >= 1e-15 && far_tol <= 0.1))) {
      set_err(c, "bad arguments to %s", name);
      throw Fail{GNK_ERR_ARG};
    }
    // a pseudo-domain of one component holding the N nodes (the even mesh
    // size only passes the domain check; the node count is N)
    gnk_domain d{};
    d.m1 = 1;
    d.n = N + (N & 1);
    d.eta = eta;
    d.etap = d.A = etap;
    const int wcols = 1 + nrhs;
    const int width = wcols >= 8 ? 8 : (wcols >= 4 ? 4 : (wcols >= 2 ? 2 : 1));
    int t, ch, sp;
    plan_pairs(c, nz, N, 16, width, false, &t, &ch, &sp);
    Batch B;
    std::vector<int64_t> off{0};
    build_batch(c, B, 1, &d, &nrhs, off, N * (int64_t)nrhs, false, false, PairShape{t, ch}, N);
    DomDev& D = B.dom[0];
    D.tz = static_cast<const double2*>(z);
    D.Nt = (int)nz;
    // treecode: the points in the Hilbert order of their positions, so that a
    // tile of consecutive targets is a compact cluster (results go back to the
    // caller's order in the epilogue)
    const int* tperm = nullptr;
    if (far_tol > 0.0) {
      std::vector<double2> hz((size_t)nz);
      HIPCHK(c, hipMemcpyAsync(hz.data(), z, sizeof(double2) * nz, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      std::vector<int> perm;
      hilbert_order(hz, perm);
      tperm = upload(c, "f_tperm", perm);
      double2* zp = ws<double2>(c, "f_zp", (size_t)nz);
      k_gather_points<<<nblocks(nz), kT, 0, c->stream>>>(static_cast<const double2*>(z), tperm, nz, zp);
      LAUNCHCHK(c);
      D.tz = zp;
    }
    D.parts = ws<double2>(c, "f_parts", (size_t)D.splits * wcols * nz);
    D.tb = ws<double4>(c, "f_tb", (size_t)((nz + 63) / 64));
    B.d_dom = upload(c, "b_dom", B.dom);
    HIPCHK(c, launch_tile_bounds(B.d_dom, 1, (int)nz, 64 * B.shape.tpt, 3, c->stream));
    k_fcau_records<<<nblocks(N), kT, 0, c->stream>>>(B.d_dom, static_cast<const double2*>(f), nrhs);
    LAUNCHCHK(c);
    if (far_tol > 0.0) build_tree(c, B, far_tol, true);
    pairs(c, B, P_SETUP, false, nullptr);
    const double2* fi = nullptr;
    if (finf) {
      const double2* h = static_cast<const double2*>(finf);
      fi = upload(c, "f_finf", std::vector<double2>(h, h + nrhs));
    }
    k_fcau_epilogue<<<dim3(nblocks(nz), (unsigned)nrhs), kT, 0, c->stream>>>(
        B.d_dom, static_cast<const double2*>(f), nrhs, fi, (double)n, tperm, static_cast<double2*>(fz));
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GNK_OK;
  }
}

gnk_status gnk_fcau(gnk_ctx* c, int64_t m1, int64_t n, const void* eta, const void* etap, const void* f, int nrhs,
                    const void* z, int64_t nz, const void* finf, void* fz) {
  return guarded(c, [&]() -> gnk_status {
    return fcau(c, "gnk_fcau", m1, n, eta, etap, f, nrhs, z, nz, finf, 0.0, fz);
  });
}

gnk_status gnk_fcau_tree(gnk_ctx* c, int64_t m1, int64_t n, const void* eta, const void* etap, const void* f,
                         int nrhs, const void* z, int64_t nz, const void* finf, double far_tol, void* fz) {
  return guarded(c, [&]() -> gnk_status {
    if (far_tol == 0.0) {
      set_err(c, "gnk_fcau_tree takes far_tol in 1e-15..0.1");
      throw Fail{GNK_ERR_ARG};
    }
    return fcau(c, "gnk_fcau_tree", m1, n, eta, etap, f, nrhs, z, nz, finf, far_tol, fz);
  });
}

gnk_status gnk_apply(gnk_ctx* c, const gnk_domain* d, int op, int prec, const double* x, int nrhs, double* y) {
  return guarded(c, [&]() -> gnk_status {
    const bool adj = (op == GNK_OP_GB || op == GNK_OP_GB_T);
    const bool unsub = (op == GNK_OP_FB_U || op == GNK_OP_GB_U);
    if (!x || !y || x == y || nrhs < 1 || op < 0 || op > GNK_OP_GB_U || (prec != GNK_FP64 && prec != GNK_MIXED)) {
      set_err(c, "bad arguments to gnk_apply");
      throw Fail{GNK_ERR_ARG};
    }
    Batch B;
    const bool mixed = prec == GNK_MIXED && op != GNK_OP_LHAT;
    single_batch(c, B, d, nrhs, adj, mixed, unsub);
    validate(c, B, x, B.T);
    if (op != GNK_OP_LHAT) {
      setup_diag(c, B);
      if (adj) setup_evec(c, B);
      if (unsub) setup_ndiag(c, B);
    }
    ApplyArgs a;
    a.mixed = mixed;
    apply_op(c, B, op, x, y, a);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GNK_OK;
  });
}

gnk_status gnk_fbie(gnk_ctx* c, const gnk_domain* d, const double* gam, int nrhs, const gnk_opts* opts, double* mu,
                    double* h, gnk_info* info) {
  return guarded(c, [&]() -> gnk_status {
    if (!gam || !mu || nrhs < 1 || mu == gam || h == gam || (h && h == mu)) {
      set_err(c, "bad arguments to gnk_fbie");
      throw Fail{GNK_ERR_ARG};
    }
    gnk_opts o = resolve_opts(c, opts);
    Batch B;
    single_batch(c, B, d, nrhs, false, o.prec == GNK_MIXED, o.no_subtraction != 0);
    if (o.far_tol > 0.0) build_tree(c, B, o.far_tol);
    GmresOut g = fbie_batch(c, B, gam, o, mu, h);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info)
      for (int r = 0; r < nrhs; ++r) info[r] = g.info[r];
    return g.all_converged ? GNK_OK : GNK_NOT_CONVERGED;
  });
}

gnk_status gnk_fbie_ad(gnk_ctx* c, const gnk_domain* d, const double* gam, int nrhs, const gnk_opts* opts, double* mu,
                       gnk_info* info) {
  return guarded(c, [&]() -> gnk_status {
    if (!gam || !mu || nrhs < 1 || mu == gam) {
      set_err(c, "bad arguments to gnk_fbie_ad");
      throw Fail{GNK_ERR_ARG};
    }
    gnk_opts o = resolve_opts(c, opts);
    Batch B;
    single_batch(c, B, d, nrhs, true, o.prec == GNK_MIXED);
    if (o.far_tol > 0.0) build_tree(c, B, o.far_tol);
    GmresOut g = fbiead_batch(c, B, gam, o, mu);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info)
      for (int r = 0; r < nrhs; ++r) info[r] = g.info[r];
    return g.all_converged ? GNK_OK : GNK_NOT_CONVERGED;
  });
}

gnk_status gnk_fbie_batched(gnk_ctx* c, int ndom, const gnk_domain* doms, const double* const* gam, const int* nrhs,
                            const gnk_opts* opts, double* const* mu, double* const* h, gnk_info* info) {
  return guarded(c, [&]() -> gnk_status {
    if (ndom < 1 || !doms || !gam || !nrhs || !mu) {
      set_err(c, "bad arguments to gnk_fbie_batched");
      throw Fail{GNK_ERR_ARG};
    }
    gnk_opts o = resolve_opts(c, opts);
    if (o.no_subtraction || o.far_tol > 0.0) {
      set_err(c, "no_subtraction and far_tol are available for gnk_fbie and gnk_fbie_ad only");
      throw Fail{GNK_ERR_ARG};
    }
    if (o.x0) {
      set_err(c, "gnk_fbie_batched takes no initial guess");
      throw Fail{GNK_ERR_ARG};
    }
    std::vector<int64_t> off(ndom);
    int64_t T = 0;
    int ncol = 0;
    for (int d = 0; d < ndom; ++d) {
      check_domain(c, &doms[d], false);
      if (nrhs[d] < 1 || !gam[d] || !mu[d]) {
        set_err(c, "domain %d: need nrhs >= 1, gam and mu", d);
        throw Fail{GNK_ERR_ARG};
      }
      off[d] = T;
      T += doms[d].m1 * doms[d].n * (int64_t)nrhs[d];
      ncol += nrhs[d];
    }
    // gather the right-hand sides into one flat vector set
    double* g = ws<double>(c, "bat_gam", T);
    double* m = ws<double>(c, "bat_mu", T);
    double* hh = h ? ws<double>(c, "bat_h", T) : nullptr;
    for (int d = 0; d < ndom; ++d)
      HIPCHK(c, hipMemcpyAsync(g + off[d], gam[d], sizeof(double) * doms[d].m1 * doms[d].n * nrhs[d],
                               hipMemcpyDeviceToDevice, c->stream));
    const bool mixed = o.prec == GNK_MIXED;
    const PairShape p = tuned_shape(c, ndom, doms, nrhs, mixed, g, off, T);
    Batch B;
    build_batch(c, B, ndom, doms, nrhs, off, T, false, mixed, p);
    GmresOut go = fbie_batch(c, B, g, o, m, hh);
    for (int d = 0; d < ndom; ++d) {
      const size_t bytes = sizeof(double) * doms[d].m1 * doms[d].n * nrhs[d];
      HIPCHK(c, hipMemcpyAsync(mu[d], m + off[d], bytes, hipMemcpyDeviceToDevice, c->stream));
      if (h && h[d]) HIPCHK(c, hipMemcpyAsync(h[d], hh + off[d], bytes, hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info)
      for (int q = 0; q < ncol; ++q) info[q] = go.info[q];
    return go.all_converged ? GNK_OK : GNK_NOT_CONVERGED;
  });
}

gnk_status gnk_fbie_adjoint(gnk_ctx* c, const gnk_domain* d, const double* g_mu, const double* g_h, int nrhs,
                            const gnk_opts* opts, double* lam, double* g_gam, gnk_info* info) {
  return guarded(c, [&]() -> gnk_status {
    if ((!g_mu && !g_h) || !lam || nrhs < 1 || lam == g_mu || lam == g_h || (g_gam && (g_gam == lam ||
        g_gam == g_mu || g_gam == g_h))) {
      set_err(c, "bad arguments to gnk_fbie_adjoint");
      throw Fail{GNK_ERR_ARG};
    }
    gnk_opts o = resolve_opts(c, opts);
    if (o.no_subtraction || o.far_tol > 0.0) {
      set_err(c, "no_subtraction and far_tol are available for gnk_fbie and gnk_fbie_ad only");
      throw Fail{GNK_ERR_ARG};
    }
    Batch B;
    single_batch(c, B, d, nrhs, false, o.prec == GNK_MIXED);
    GmresOut g = fbie_adjoint_batch(c, B, g_mu, g_h, o, lam, g_gam);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info)
      for (int r = 0; r < nrhs; ++r) info[r] = g.info[r];
    return g.all_converged ? GNK_OK : GNK_NOT_CONVERGED;
  });
}

gnk_status gnk_geom_vjp(gnk_ctx* c, const gnk_domain* d, int nterms, const int* ops, const double* coef,
                        const double* const* u, const double* const* v, void* g_eta, void* g_etap, void* g_A) {
  return guarded(c, [&]() -> gnk_status {
    bool ok = nterms >= 1 && nterms <= 64 && ops && u && v && (g_eta || g_etap || g_A);
    for (int t = 0; ok && t < nterms; ++t)
      ok = (ops[t] == GNK_OP_FB || ops[t] == GNK_OP_FC) && u[t] && v[t] && (!coef || std::isfinite(coef[t]));
    if (ok && d) {
      const void* in[3] = {d->eta, d->etap, d->A};
      const void* out[3] = {g_eta, g_etap, g_A};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) ok = ok && (!out[b] || out[b] != in[a]);
    }
    if (!ok) {
      set_err(c, "bad arguments to gnk_geom_vjp");
      throw Fail{GNK_ERR_ARG};
    }
    geom_vjp(c, d, nterms, ops, coef, u, v, static_cast<double2*>(g_eta), static_cast<double2*>(g_etap),
             static_cast<double2*>(g_A));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GNK_OK;
  });
}

namespace {
bool fourier_args_ok(int64_t m1, int64_t n, int kmin, int nk) {
  return m1 >= 1 && m1 <= 65535 && n >= 1 && m1 * n <= ((int64_t)1 << 30) && nk >= 1 && nk <= 65535 &&
         kmin >= -(1 << 20) && (int64_t)kmin + nk <= (1 << 20);
}
}  // namespace

gnk_status gnk_fourier_curve(gnk_ctx* c, int64_t m1, int64_t n, int kmin, int nk, int ccw, const void* coef,
                             void* eta, void* etap, void* etapp) {
  return guarded(c, [&]() -> gnk_status {
    if (!fourier_args_ok(m1, n, kmin, nk) || !coef || !eta || coef == eta || (etap && (etap == eta || etap == coef)) ||
        (etapp && (etapp == eta || etapp == coef || etapp == etap))) {
      set_err(c, "bad arguments to gnk_fourier_curve");
      throw Fail{GNK_ERR_ARG};
    }
    HIPCHK(c, launch_fourier_curve(static_cast<const double2*>(coef), (int)m1, (int)n, kmin, nk, ccw ? 1 : -1,
                                   static_cast<double2*>(eta), static_cast<double2*>(etap),
                                   static_cast<double2*>(etapp), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GNK_OK;
  });
}

gnk_status gnk_fourier_vjp(gnk_ctx* c, int64_t m1, int64_t n, int kmin, int nk, int ccw, const void* g_eta,
                           const void* g_etap, const void* g_etapp, void* g_coef) {
  return guarded(c, [&]() -> gnk_status {
    if (!fourier_args_ok(m1, n, kmin, nk) || !g_coef || (!g_eta && !g_etap && !g_etapp) || g_coef == g_eta ||
        g_coef == g_etap || g_coef == g_etapp) {
      set_err(c, "bad arguments to gnk_fourier_vjp");
      throw Fail{GNK_ERR_ARG};
    }
    HIPCHK(c, launch_fourier_vjp(static_cast<const double2*>(g_eta), static_cast<const double2*>(g_etap),
                                 static_cast<const double2*>(g_etapp), (int)m1, (int)n, kmin, nk, ccw ? 1 : -1,
                                 static_cast<double2*>(g_coef), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GNK_OK;
  });
}

}  // extern "C"

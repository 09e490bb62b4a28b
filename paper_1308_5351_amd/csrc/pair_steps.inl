// Direct pair loops shared by the FP64 pair kernels (one reciprocal per one,
// two or four sources), included inside gnk's anonymous namespace.
#pragma once

template <int NR, int TPT>
struct Acc {
  double x[TPT][NR];
  double y[TPT][NR];
};

// acc[t] += w * q for NR columns, q = conj(d)/|d|^2 = (qx, qy)
template <int NR, int TPT, class P>
__device__ __forceinline__ void accumulate(Acc<NR, TPT>& a, int t, P wj, double qx, double qy) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double2 w = wj[r];
    a.x[t][r] = __builtin_fma(w.x, qx, a.x[t][r]);
    a.x[t][r] = __builtin_fma(-w.y, qy, a.x[t][r]);
    a.y[t][r] = __builtin_fma(w.x, qy, a.y[t][r]);
    a.y[t][r] = __builtin_fma(w.y, qx, a.y[t][r]);
  }
}

// two sources a, b (records ra, rb) against every target of the lane
// ra, rb: source records (eta at [0]); the launch's weight columns start at [wo]
template <int NR, int TPT, class P>
__device__ __forceinline__ void pair_step(Acc<NR, TPT>& acc, const double2 (&tg)[TPT], P ra, P rb, int wo) {
  const double2 ea = ra[0], eb = rb[0];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const double dxa = tg[t].x - ea.x, dya = tg[t].y - ea.y;
    const double dxb = tg[t].x - eb.x, dyb = tg[t].y - eb.y;
    const double da = __builtin_fma(dya, dya, dxa * dxa);
    const double db = __builtin_fma(dyb, dyb, dxb * dxb);
    const double R = refine_rcp(da * db);
    const double qa = db * R, qb = da * R;
    accumulate<NR, TPT>(acc, t, ra + wo, dxa * qa, -dya * qa);
    accumulate<NR, TPT>(acc, t, rb + wo, dxb * qb, -dyb * qb);
  }
}

// four sources a..d against every target of the lane, one reciprocal for all
// four: with R = 1/(|da|^2 |db|^2 |dc|^2 |dd|^2), 1/|da|^2 = R |db|^2 (|dc|^2 |dd|^2)
// and so on (the product stays in range while every distance lies in
// [1e-38, 1e38])
template <int NR, int TPT, class P>
__device__ __forceinline__ void quad_step(Acc<NR, TPT>& acc, const double2 (&tg)[TPT], P ra, P rb, P rc, P rd,
                                          int wo) {
  const double2 ea = ra[0], eb = rb[0], ec = rc[0], ed = rd[0];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const double dxa = tg[t].x - ea.x, dya = tg[t].y - ea.y;
    const double dxb = tg[t].x - eb.x, dyb = tg[t].y - eb.y;
    const double dxc = tg[t].x - ec.x, dyc = tg[t].y - ec.y;
    const double dxd = tg[t].x - ed.x, dyd = tg[t].y - ed.y;
    const double da = __builtin_fma(dya, dya, dxa * dxa);
    const double db = __builtin_fma(dyb, dyb, dxb * dxb);
    const double dc = __builtin_fma(dyc, dyc, dxc * dxc);
    const double dd = __builtin_fma(dyd, dyd, dxd * dxd);
    const double ab = da * db, cd = dc * dd;
    const double R = refine_rcp(ab * cd);
    const double Rab = R * cd, Rcd = R * ab;
    const double qa = db * Rab, qb = da * Rab, qc = dd * Rcd, qd = dc * Rcd;
    accumulate<NR, TPT>(acc, t, ra + wo, dxa * qa, -dya * qa);
    accumulate<NR, TPT>(acc, t, rb + wo, dxb * qb, -dyb * qb);
    accumulate<NR, TPT>(acc, t, rc + wo, dxc * qc, -dyc * qc);
    accumulate<NR, TPT>(acc, t, rd + wo, dxd * qd, -dyd * qd);
  }
}

template <int NR, int TPT, class P>
__device__ __forceinline__ void single_step(Acc<NR, TPT>& acc, const double2 (&tg)[TPT], const int (&ti)[TPT], P rj,
                                            int wo, int j, bool masked) {
  const double2 e = rj[0];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const double dx = tg[t].x - e.x, dy = tg[t].y - e.y;
    double r = refine_rcp(__builtin_fma(dy, dy, dx * dx));
    if (masked) r = (j == ti[t]) ? 0.0 : r;
    accumulate<NR, TPT>(acc, t, rj + wo, dx * r, -dy * r);
  }
}

// One source record held in scalar registers: its node and the launch's NR
// weight columns.
template <int NR>
struct SrcRec {
  double2 e;
  double2 w[NR];
};

template <int NR, class P>
__device__ __forceinline__ void load_src(SrcRec<NR>& s, P r, int wo) {
  s.e = r[0];
#pragma unroll
  for (int q = 0; q < NR; ++q) s.w[q] = r[wo + q];
}

// Source s against every target of the lane (TPT even). The lane's targets
// are taken in twos that share one reciprocal: with R = 1/(|d0|^2 |d1|^2),
// 1/|d0|^2 = R |d1|^2 and 1/|d1|^2 = R |d0|^2. The record of the following
// source is loaded into nx (from rn) only after s has first been used: scalar
// loads may return out of order, so the wait before a use of s covers every
// scalar load issued before it, and a load issued earlier would be waited for
// at once instead of during this step's arithmetic.
template <int NR, int TPT, class P>
__device__ __forceinline__ void stream_step(Acc<NR, TPT>& acc, const double2 (&tg)[TPT], const SrcRec<NR>& s,
                                            SrcRec<NR>& nx, P rn, int wo) {
  double dx[TPT], dy[TPT];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    dx[t] = tg[t].x - s.e.x;
    dy[t] = tg[t].y - s.e.y;
  }
  __builtin_amdgcn_sched_barrier(0);
  load_src<NR>(nx, rn, wo);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int t = 0; t < TPT; t += 2) {
    const double d0 = __builtin_fma(dy[t], dy[t], dx[t] * dx[t]);
    const double d1 = __builtin_fma(dy[t + 1], dy[t + 1], dx[t + 1] * dx[t + 1]);
    const double R = refine_rcp(d0 * d1);
    const double q0 = d1 * R, q1 = d0 * R;
    const double qx[2] = {dx[t] * q0, dx[t + 1] * q1};
    const double qy[2] = {-dy[t] * q0, -dy[t + 1] * q1};
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double2 w = s.w[r];
        acc.x[t + u][r] = __builtin_fma(w.x, qx[u], acc.x[t + u][r]);
        acc.x[t + u][r] = __builtin_fma(-w.y, qy[u], acc.x[t + u][r]);
        acc.y[t + u][r] = __builtin_fma(w.x, qy[u], acc.y[t + u][r]);
        acc.y[t + u][r] = __builtin_fma(w.y, qx[u], acc.y[t + u][r]);
      }
  }
}

// Sources [ja, jb) (none of them a target of the lane) one at a time, the
// next record in flight while the current one is summed: the near tiles of
// 8-column mixed products (short runs of 64 sources between tile tests), whose
// two records per step would fill the scalar registers and leave no room to
// load ahead. The last prefetch re-reads source jb - 1.
template <int NR, int TPT, class P>
__device__ __forceinline__ void stream_range(Acc<NR, TPT>& acc, const double2 (&tg)[TPT], P rec, int stride, int wo,
                                             int ja, int jb) {
  static_assert(TPT % 2 == 0, "targets are paired");
  if (ja >= jb) return;
  SrcRec<NR> a, b;
  load_src<NR>(a, rec + (size_t)ja * stride, wo);
  int j = ja;
  for (; j + 1 < jb; j += 2) {
    stream_step<NR, TPT>(acc, tg, a, b, rec + (size_t)(j + 1) * stride, wo);
    stream_step<NR, TPT>(acc, tg, b, a, rec + (size_t)min(j + 2, jb - 1) * stride, wo);
  }
  if (j < jb) stream_step<NR, TPT>(acc, tg, a, b, rec + (size_t)j * stride, wo);
}

// Two sources a, b against the lane's targets taken in twos (TPT even), one
// reciprocal for the four pairs: with P_t = |da_t|^2 |db_t|^2 and
// R = 1/(P_0 P_1), 1/|da_0|^2 = R P_1 |db_0|^2 and so on (the product stays in
// range while every squared distance lies in [1e-75, 1e75]).
template <int NR, int TPT, class P>
__device__ __forceinline__ void pair_step_t2(Acc<NR, TPT>& acc, const double2 (&tg)[TPT], P ra, P rb, int wo) {
  static_assert(TPT % 2 == 0, "targets are paired");
  const double2 ea = ra[0], eb = rb[0];
#pragma unroll
  for (int t = 0; t < TPT; t += 2) {
    double dxa[2], dya[2], dxb[2], dyb[2], da[2], db[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      dxa[u] = tg[t + u].x - ea.x;
      dya[u] = tg[t + u].y - ea.y;
      dxb[u] = tg[t + u].x - eb.x;
      dyb[u] = tg[t + u].y - eb.y;
      da[u] = __builtin_fma(dya[u], dya[u], dxa[u] * dxa[u]);
      db[u] = __builtin_fma(dyb[u], dyb[u], dxb[u] * dxb[u]);
    }
    const double p0 = da[0] * db[0], p1 = da[1] * db[1];
    const double R = refine_rcp(p0 * p1);
    const double r[2] = {R * p1, R * p0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const double qa = db[u] * r[u], qb = da[u] * r[u];
      accumulate<NR, TPT>(acc, t + u, ra + wo, dxa[u] * qa, -dya[u] * qa);
      accumulate<NR, TPT>(acc, t + u, rb + wo, dxb[u] * qb, -dyb[u] * qb);
    }
  }
}

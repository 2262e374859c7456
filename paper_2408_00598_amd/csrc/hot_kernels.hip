// HIP kernels of the HOT iteration (arXiv 2408.00598, Algorithm 2) for gfx950.
//
// One iteration is three launches (the first in hot_slab.hip):
//   k_slab_pass   streams every slab of the flow state once (Steps 2-4 fused:
//                 g = c - A^T ybar, shat = |s - 2g|, Halpern step) and produces
//                 the row / column sums of the new state (the A s of Step 1 of
//                 the next iteration) and, on check passes, the partial sums of
//                 the relative KKT residual (eq. kkt_res).
//   k_pair_reduce assembles R = b/sigma - A(s - c) from those sums and the
//                 block sums the structured solve needs.
//   k_pair_solve  decides stop / restart on check passes and solves
//                 A A^T ybar = R (Prop. 3) in O(M), writing the per-slab
//                 alpha / beta vectors the next slab pass reads.
// Reductions have a fixed order (no floating-point atomics), so a problem
// gives bit-identical results alone or inside a batch.
#include "hot_device.h"
#include "hot_internal.h"
#include "hot_runtime.h"

#include <algorithm>

namespace hot {

void launch_slab_pass(const LaunchArgs& a, int par, hipStream_t st);

// ---------------------------------------------------------------------------
// Pair reduce: R = b/sigma - A(s - c) from the slab sums, the totals the
// structured solve needs, and (check passes) the KKT partials.  Four block
// kinds, so that rows of both families run on separate waves:
//   kind 0, F1 row block b (slot b): one wave per row j = 4b + w of R2 and
//           the total of row j of the F1 row sums;
//   kind 3, F2 row block b (slot nb1 + b): one wave per row k = 4b + w of
//           R3^T and the total of row k of the F2 row sums;
//   kind 1, strip s: u1[k] = sum_j rs1[j][k] for 64 columns k (lane per column);
//   kind 2, strip s: u2[j] = sum_k rs2[k][j] for 64 columns j.
// A family with slab side >= kWideSide ("wide") instead gives each row a
// whole block (row j = b or k = b, the 256 threads over its columns), so a
// large pair spreads its column-partial sums over four times the waves.
// Column sums of a slab arrive as per-chunk partials; they are added with
// four independent accumulators (fixed order) so the loads overlap.
// R1 itself is never stored: the solve reads it straight from the two
// row-sum arrays, tile by tile.
// With C_L(p) = sum_q (X_p - X_q)^2 and CC_L = sum_p C_L(p) from the family's
// cost table (X_p = p on the uniform grid):
//   R1[j][k] = -(rs1[j][k] - C_m(k)) + (rs2[k][j] - C_n(j)),
//   1^T R1^j = -(tot1[j] - CC_m) + (u2[j] - m C_n(j)),
//   sum_j R1[j][k] = -(u1[k] - n C_m(k)) + (tot2[k] - CC_n).
// ---------------------------------------------------------------------------
__device__ inline double dinv(int m, int k) { return (k == m - 1) ? 1.0 / (m + 1.0) : 1.0 / m; }

// sum_c p[c * stride], c < nchunk, in a fixed order with four accumulators
// (non-temporal loads: column partials are streamed once per use; -13% on
// the 512x512 reduce)
__device__ inline double chunk_sum(const double* __restrict__ p, int nchunk, int64_t stride) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int c = 0;
  for (; c + 4 <= nchunk; c += 4) {
    a0 += __builtin_nontemporal_load(p + (int64_t)c * stride);
    a1 += __builtin_nontemporal_load(p + (int64_t)(c + 1) * stride);
    a2 += __builtin_nontemporal_load(p + (int64_t)(c + 2) * stride);
    a3 += __builtin_nontemporal_load(p + (int64_t)(c + 3) * stride);
  }
  for (; c < nchunk; ++c) a0 += __builtin_nontemporal_load(p + (int64_t)c * stride);
  return (a0 + a1) + (a2 + a3);
}

// chunk_sum of two columns at once (q is read only when `two`): the same
// order per column, twice the loads in flight
__device__ inline void chunk_sum2(const double* __restrict__ p, const double* __restrict__ q,
                                  bool two, int nchunk, int64_t stride, double& s0,
                                  double& s1) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
  int c = 0;
  for (; c + 4 <= nchunk; c += 4) {
    a0 += __builtin_nontemporal_load(p + (int64_t)c * stride);
    a1 += __builtin_nontemporal_load(p + (int64_t)(c + 1) * stride);
    a2 += __builtin_nontemporal_load(p + (int64_t)(c + 2) * stride);
    a3 += __builtin_nontemporal_load(p + (int64_t)(c + 3) * stride);
    if (two) {
      b0 += __builtin_nontemporal_load(q + (int64_t)c * stride);
      b1 += __builtin_nontemporal_load(q + (int64_t)(c + 1) * stride);
      b2 += __builtin_nontemporal_load(q + (int64_t)(c + 2) * stride);
      b3 += __builtin_nontemporal_load(q + (int64_t)(c + 3) * stride);
    }
  }
  for (; c < nchunk; ++c) {
    a0 += __builtin_nontemporal_load(p + (int64_t)c * stride);
    if (two) b0 += __builtin_nontemporal_load(q + (int64_t)c * stride);
  }
  s0 = (a0 + a1) + (a2 + a3);
  s1 = (b0 + b1) + (b2 + b3);
}

// block-wide fixed-order totals of q values held by lane 0 of each wave
__device__ inline double wave4(const double (&w)[4][kKP], int q) {
  return (w[0][q] + w[1][q]) + (w[2][q] + w[3][q]);
}

// One reduce block's work (the body of k_pair_reduce, also the reduce role
// of k_pair_fused).
__device__ __forceinline__ void reduce_block(
    const PBlock pbk, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, const double* __restrict__ rowsum,
    const double* __restrict__ colpart, const double* __restrict__ rowsum_prev,
    const double* __restrict__ colpart_prev, const double* __restrict__ kitem,
    const double* __restrict__ ab, double* __restrict__ abY, double* __restrict__ arr,
    double* __restrict__ vec, unsigned long long* __restrict__ bytes_ctr, int elem) {
  __shared__ double wred[4][kKP];
  __shared__ double strip[4][64];
  __shared__ double blk_red[4];
  const PairCtl* cp = ctl + pbk.pair;
  if (cp->status != ST_RUNNING) return;
  const int mode = cp->mode;
  if (mode == MODE_IDLE) return;
  const PairGeo G = geo[pbk.pair];
  const int m = G.m, n = G.n, b = pbk.blk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const FamGeo F1 = G.f[0], F2 = G.f[1];
  if (bytes_ctr && pbk.kind == 0 && b == 0 && threadIdx.x == 0 && mode != MODE_INIT) {
    // measurement only: algorithmic bytes of the slab pass this pair just
    // had -- read the state (and the anchor when it is a buffer of its own),
    // write the new state; with sigma re-balancing also read (check) or
    // write (restart) x_bar of the last restart; padding excluded
    const bool sep = mode != MODE_RESTART && cp->anc >= 0 && cp->anc != cp->src;
    const bool xr = (cp->flags & 0x10) && (mode == MODE_CHECK || mode == MODE_RESTART);
    const unsigned long long N = (unsigned long long)m * m * n + (unsigned long long)m * n * n;
    atomicAdd(bytes_ctr, N * (unsigned long long)elem * (2ull + (sep ? 1 : 0) + (xr ? 1 : 0)));
  }
  if (pbk.kind == 1 || pbk.kind == 2) {
    // column totals of a row-sum array: lane = column, waves split the rows
    const bool s1 = pbk.kind == 1;
    const int ncol = s1 ? m : n, nrow = s1 ? n : m;
    const double* rs = s1 ? rowsum + F1.rsoff : rowsum + F2.rsoff;  // [nrow][ncol]
    const int col = 64 * b + lane;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (col < ncol) {
      int r = wave;
      for (; r + 12 < nrow; r += 16) {
        a0 += rs[(int64_t)r * ncol + col];
        a1 += rs[(int64_t)(r + 4) * ncol + col];
        a2 += rs[(int64_t)(r + 8) * ncol + col];
        a3 += rs[(int64_t)(r + 12) * ncol + col];
      }
      for (; r < nrow; r += 4) a0 += rs[(int64_t)r * ncol + col];
    }
    strip[wave][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (wave == 0) {
      const double tot = (strip[0][lane] + strip[1][lane]) + (strip[2][lane] + strip[3][lane]);
      double pu = 0.0;
      if (col < ncol) {
        vec[(s1 ? vec_u1(G) : vec_u2(G)) + col] = tot;
        if (s1) pu = (-(tot - (double)n * fam_cr(ab, F1, col))) * dinv(m, col);
      }
      if (s1) {
        pu = wave_sum(pu);
        if (lane == 0) {
          double* sp = vec + vec_spart(G) + 4 * (int64_t)(G.nblk + b);
          sp[0] = 0.0;
          sp[1] = 0.0;
          sp[2] = pu;
        }
      }
    }
    return;
  }
  const bool f1 = pbk.kind == 0;
  // narrow family: slot q holds rows 4q..4q+3 (wave w takes row 4q + w, its
  // lanes the columns) and a block takes rq consecutive slots; wide family
  // (large slabs): slot q is row q alone, its block's 256 threads the columns
  const bool wide = (f1 ? F1.wide : F2.wide) != 0;
  const int nq = wide ? 1 : G.rq;
  const int nslot = f1 ? G.nb1 : G.nblk - G.nb1;
  for (int qd = 0; qd < nq; ++qd) {
    const int sq = nq * b + qd;  // slot within the family
    if (sq >= nslot) break;
    if (qd > 0) __syncthreads();  // the previous slot's wred has been read
    const int slot = f1 ? sq : G.nb1 + sq;
    const int r = wide ? sq : 4 * sq + wave;  // row j (F1 block) or k (F2 block)
    const int tid = wide ? (int)threadIdx.x : lane;
    const int nthr = wide ? kWG : 64;
    const bool lead = tid == 0;             // writes the slab's totals
    // a slab total: over the wave, or over the block for a wide family (every
    // thread of the block calls it then)
    auto slab_sum = [&](double v) { return wide ? block_sum(v, blk_red) : wave_sum(v); };
    const double isg = 1.0 / cp->sigma;
    const double* mu1T = arr + arr_mu1T(G);
    const double* mu2 = arr + arr_mu2(G);
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;  // (sum a_j, sum PR3, sum Sp / D) partials
    if (f1 && r < n) {
      const int j = r;
      double* R2 = arr + arr_R2(G);
      double sr2 = 0.0, t1 = 0.0;
      const double* cpj = colpart + F1.cpoff + (int64_t)j * F1.nchunk * m;
      // columns tid, tid + nthr, ... in that order, two per step
      for (int i0 = tid; i0 < m; i0 += 2 * nthr) {
        double cs[2];
        chunk_sum2(cpj + i0, cpj + i0 + nthr, i0 + nthr < m, F1.nchunk, m, cs[0], cs[1]);
        for (int h = 0; h < 2; ++h) {
          const int i = i0 + h * nthr;
          if (i >= m) break;
          const double r2 = mu1T[(int64_t)j * m + i] * isg - (cs[h] - fam_cr(ab, F1, i));
          R2[(int64_t)j * m + i] = r2;
          sr2 += r2;
          t1 += rowsum[F1.rsoff + (int64_t)j * m + i];  // row j of the F1 row sums
        }
      }
      sr2 = slab_sum(sr2);
      t1 = slab_sum(t1);
      if (lead) {
        vec[vec_a(G) + j] = sr2;
        vec[vec_tot1(G) + j] = t1;
      }
      p0 = sr2;
    } else if (!f1 && r < m) {
      const int k = r;
      double* R3T = arr + arr_R3T(G);
      double s3 = 0.0, t2 = 0.0;
      const double* cpk = colpart + F2.cpoff + (int64_t)k * F2.nchunk * n;
      for (int l0 = tid; l0 < n; l0 += 2 * nthr) {
        double cs[2];
        chunk_sum2(cpk + l0, cpk + l0 + nthr, l0 + nthr < n, F2.nchunk, n, cs[0], cs[1]);
        for (int h = 0; h < 2; ++h) {
          const int l = l0 + h * nthr;
          if (l >= n) break;
          double r3 = 0.0;
          if (!(k == m - 1 && l == n - 1))
            r3 = mu2[(int64_t)k * n + l] * isg - (cs[h] - fam_cr(ab, F2, l));
          R3T[(int64_t)k * n + l] = r3;
          s3 += r3;
          t2 += rowsum[F2.rsoff + (int64_t)k * n + l];  // row k of the F2 row sums
        }
      }
      s3 = slab_sum(s3);
      t2 = slab_sum(t2);
      if (lead) {
        vec[vec_PR3(G) + k] = s3;
        vec[vec_tot2(G) + k] = t2;
      }
      p1 = s3;
      p2 = ((t2 - fam_cc(ab, F2)) + s3) * dinv(m, k);
    }
    if (wide && wave != 0) p0 = p1 = p2 = 0.0;  // (every wave holds the slab totals)
    if (lane == 0) {
      wred[wave][0] = p0;
      wred[wave][1] = p1;
      wred[wave][2] = p2;
    }
    __syncthreads();
    if (threadIdx.x < 3)
      vec[vec_spart(G) + 4 * (int64_t)slot + threadIdx.x] = wave4(wred, threadIdx.x);
    const bool su = (cp->flags & 0x10) != 0;
    // (alpha, beta) of this block's slab and their stored copy from the last restart
    const FamGeo& FS = f1 ? F1 : F2;
    const int LS = f1 ? m : n;
    const bool has_slab = f1 ? r < n : r < m;
    const int64_t aoff = FS.aboff + (int64_t)r * 2 * LS;
    if (mode == MODE_RESTART && su && has_slab) {
      // sigma re-balancing: keep y_bar of this restart (alpha, beta, their sums)
      for (int q = tid; q < 2 * LS; q += nthr) abY[aoff + q] = ab[aoff + q];
      if (tid < 2) abY[FS.sumoff + 2 * (int64_t)r + tid] = ab[FS.sumoff + 2 * (int64_t)r + tid];
    }
    if (mode != MODE_CHECK) continue;

    // ---- check pass: KKT partials of w_bar^k -------------------------------
    double part[kNKP] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    {
      const int i0 = G.item0 + slot * G.ipb;
      const int i1 = min(G.item0 + G.nitem, i0 + G.ipb);
      for (int it = i0 + (int)threadIdx.x; it < i1; it += kWG)
        for (int q = 0; q <= KI_DX; ++q) part[q] += kitem[(int64_t)it * kKI + q];
    }
    if (su && has_slab) {
      // ||A^T (y_bar - Y)||^2 over this slab: A^T y is alpha_p + beta_q on it,
      // so the sum over the L x L slab is L sum da^2 + L sum db^2 + 2 sum da sum db
      double a2 = 0.0, b2 = 0.0, sa_ = 0.0, sb_ = 0.0;
      for (int q = tid; q < LS; q += nthr) {
        const double da = ab[aoff + q] - abY[aoff + q];
        const double db = ab[aoff + LS + q] - abY[aoff + LS + q];
        a2 += da * da;
        b2 += db * db;
        sa_ += da;
        sb_ += db;
      }
      a2 = slab_sum(a2);
      b2 = slab_sum(b2);
      sa_ = slab_sum(sa_);
      sb_ = slab_sum(sb_);
      if (lead) part[KP_DY] = (double)LS * (a2 + b2) + 2.0 * sa_ * sb_;
    }
    // primal residual A xbar - b, xbar = sigma (s - g): the sums of s^k are the
    // previous pass's sums; the sums of g over a slab row / column follow from
    // alpha, beta and their per-slab totals.
    const double sg = cp->sigma;
    double prim = 0.0, by = 0.0;
    if (f1 && r < n) {
      const int j = r;
      const double* al = ab + F1.aboff + (int64_t)j * 2 * m;
      const double* be = al + m;
      const double sa = ab[F1.sumoff + 2 * (int64_t)j], sb = ab[F1.sumoff + 2 * (int64_t)j + 1];
      for (int kk = tid; kk < m; kk += nthr) {
        // row kk of F1^(j) and row j of F2^(kk) share the conservation row (j,kk)
        const double* al2 = ab + F2.aboff + (int64_t)kk * 2 * n;
        const double sb2 = ab[F2.sumoff + 2 * (int64_t)kk + 1];
        const double x1 = sg * (rowsum_prev[F1.rsoff + (int64_t)j * m + kk] -
                                (fam_cr(ab, F1, kk) - m * al[kk] - sb));
        const double x2 = sg * (rowsum_prev[F2.rsoff + (int64_t)kk * n + j] -
                                (fam_cr(ab, F2, j) - n * al2[j] - sb2));
        const double rr = x1 - x2;
        prim += rr * rr;
      }
      const double* cpj = colpart_prev + F1.cpoff + (int64_t)j * F1.nchunk * m;
      for (int i = tid; i < m; i += nthr) {
        const double cs = chunk_sum(cpj + i, F1.nchunk, m);
        const double x = sg * (cs - (fam_cr(ab, F1, i) - sa - m * be[i]));
        const double rr = x - mu1T[(int64_t)j * m + i];
        prim += rr * rr;
        by += mu1T[(int64_t)j * m + i] * be[i];
      }
    } else if (!f1 && r < m) {
      const int k = r;
      const double* al = ab + F2.aboff + (int64_t)k * 2 * n;
      const double* be = al + n;
      const double sa = ab[F2.sumoff + 2 * (int64_t)k];
      const double* cpk = colpart_prev + F2.cpoff + (int64_t)k * F2.nchunk * n;
      for (int l = tid; l < n; l += nthr) {
        if (k == m - 1 && l == n - 1) continue;
        const double cs = chunk_sum(cpk + l, F2.nchunk, n);
        const double x = sg * (cs - (fam_cr(ab, F2, l) - sa - n * be[l]));
        const double rr = x - mu2[(int64_t)k * n + l];
        prim += rr * rr;
        by += mu2[(int64_t)k * n + l] * be[l];
      }
    }
    part[KP_PRIM] = prim;
    part[KP_BY] = by;
    __syncthreads();
    for (int q = 0; q < kNKP; ++q) {
      const double v = wave_sum(part[q]);
      if (lane == 0) wred[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kNKP)
      vec[vec_kpart(G) + (int64_t)slot * kKP + threadIdx.x] = wave4(wred, threadIdx.x);
  }
}

__global__ __launch_bounds__(kWG) void k_pair_reduce(
    const PBlock* __restrict__ blocks, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, const double* __restrict__ rowsum,
    const double* __restrict__ colpart, const double* __restrict__ rowsum_prev,
    const double* __restrict__ colpart_prev, const double* __restrict__ kitem,
    const double* __restrict__ ab, double* __restrict__ abY, double* __restrict__ arr,
    double* __restrict__ vec, unsigned long long* __restrict__ bytes_ctr, int elem) {
  reduce_block(blocks[blockIdx.x], geo, ctl, rowsum, colpart, rowsum_prev, colpart_prev, kitem,
               ab, abY, arr, vec, bytes_ctr, elem);
}

// ---------------------------------------------------------------------------
// Decision after a pass (taken by one wave of every solve block of the pair,
// on identical data, so all blocks agree).
// ---------------------------------------------------------------------------
// KKT partials of a pair reduced by one wave (fixed lane-strided order, then a
// butterfly); every lane returns the totals.
__device__ inline void reduce_kpart(const PairGeo& G, const double* vec, int lane, double* acc) {
  const double* kp = vec + vec_kpart(G);
  for (int q = 0; q < kNKP; ++q) {
    double v = 0.0;
    for (int b = lane; b < G.nblk; b += 64) v += kp[(int64_t)b * kKP + q];
    acc[q] = wave_sum(v);
  }
}

__device__ void decide(const PairGeo& G, const PairCtl& c, const double* acc, PairCtl& nx,
                       bool& solve) {
  nx = c;
  solve = false;
  const bool fixed = (c.flags & 2) != 0;
  const bool admm = (c.flags & 4) != 0;
  const bool restart_on = (c.flags & 1) != 0 && !fixed && !admm;
  switch (c.mode) {
    case MODE_INIT:
      nx.k = 0;
      nx.it = 0;
      nx.src = 0;
      nx.anc = -1;
      solve = true;
      break;
    case MODE_NORMAL:
      nx.k = c.k + 1;
      nx.it = c.it + 1;
      nx.src = c.dst;
      solve = true;
      break;
    case MODE_RESTART:
      nx.k = 0;
      nx.src = 2;
      nx.anc = 2;
      solve = true;
      break;
    case MODE_CHECK: {
      const double nx2 = sqrt(acc[KP_XX]), nz2 = sqrt(acc[KP_ZZ]);
      nx.res_d = sqrt(acc[KP_DUAL]) / (1.0 + G.norm_c);
      nx.res_c = sqrt(acc[KP_COMP]) / (1.0 + nx2 + nz2);
      nx.res_p = sqrt(acc[KP_PRIM]) / (1.0 + G.norm_b);
      nx.kkt = fmax(nx.res_d, fmax(nx.res_c, nx.res_p));
      nx.kkt_abs = sqrt(acc[KP_PRIM] + acc[KP_COMP] + acc[KP_DUAL]);
      const double crit = (c.flags & 8) ? nx.kkt_abs : nx.kkt;
      nx.pobj = acc[KP_CX];
      nx.dobj = acc[KP_BY];
      nx.fp_res = sqrt(acc[KP_FP]);
      const double r = nx.fp_res;
      if (fixed) {  // metrics of w_bar^K only; s^K stays in src
        nx.status = ST_FIXED_DONE;
        nx.mode = MODE_IDLE;
        return;
      }
      if (!isfinite(nx.kkt) || !isfinite(r) || !isfinite(nx.pobj)) {
        nx.status = ST_NUMERIC;
      } else if (c.tol > 0 && crit <= c.tol) {
        nx.status = ST_CONVERGED;
      } else if (c.it >= c.max_iter) {
        nx.status = ST_MAXITER;
      } else {
        bool do_restart = false;
        if (restart_on) {
          if (c.k == 0) {
            nx.r_start = r;
            nx.r_prev = r;
          } else if (r <= 0.2 * c.r_start || (r <= 0.8 * c.r_start && r > c.r_prev)) {
            do_restart = true;
          } else {
            nx.r_prev = r;
          }
        }
        if (do_restart) {
          nx.mode = MODE_RESTART;
          nx.it = c.it + 1;
          nx.restarts = c.restarts + 1;
          nx.k = 0;
          nx.sig_old = c.sigma;
          if (c.flags & 0x10) {
            // sigma re-balancing: ||x_bar - X|| / ||A^T (y_bar - Y)|| over the
            // epoch that ends here; the restart pass writes x_bar / sigma_new
            // + z_bar, and the reduce of that pass already uses sigma_new
            const double dx = sqrt(acc[KP_DX]), dy = sqrt(acc[KP_DY]);
            if (dx > 0.0 && dy > 0.0 && isfinite(dx / dy)) nx.sigma = dx / dy;
          }
          return;  // src keeps s^k for the restart pass
        }
        nx.k = c.k + 1;
        nx.it = c.it + 1;
        nx.src = c.dst;
        solve = true;
      }
      break;
    }
    default:
      break;
  }
  if (nx.status != ST_RUNNING) return;
  // Halpern weight 1/(k+2) toward the epoch's anchor; for the ADMM baseline
  // s <- (1 - rho) s + rho s_bar = (1 - rho/2) s + (rho/2) shat, i.e. the
  // anchor is the current state itself with weight 1 - rho/2
  nx.lam = admm ? 1.0 - 0.5 * c.relax : 1.0 / (double)(nx.k + 2);
  // fixed mode: plain updates, then one check pass at it == K that only
  // evaluates w_bar^K
  nx.mode = fixed ? (nx.it >= c.max_iter ? MODE_CHECK : MODE_NORMAL)
                  : ((nx.k % c.T == 0 || nx.it >= c.max_iter) ? MODE_CHECK : MODE_NORMAL);
  const bool pingpong = (c.flags & 0x100) != 0;  // never update the state in place
  nx.dst = (pingpong || nx.mode == MODE_CHECK || nx.src == 2) ? (nx.src == 0 ? 1 : 0) : nx.src;
  if (admm) nx.anc = nx.src;
  // timing runs of the autotuner (fixed iterations only): the anchor is a
  // zero buffer of its own, so passes stream three vectors as after a restart
  if (c.flags & 0x200) nx.anc = 2;
}

// ---------------------------------------------------------------------------
// Structured solve of A A^T ybar = R (Prop. 3), Schur complement on y1:
//   Rhat1^j = R1^j - (1^T R2^j / m) 1 + PR3 / n,   S = sum_j Rhat1^j,
//   (D - 1 1^T) t = S,  D = diag(m, .., m, m+1),   t = sum_j y1^j,
//   t = D^{-1} S + m(m+1) (1^T D^{-1} S) D^{-1} 1   (Sherman-Morrison),
//   y1^j = (I + 1 1^T / n)(Rhat1^j + Q t)/(m+n),  Q = I - e_m e_m^T / n,
//   y2^j = (R2^j - (1^T y1^j) 1)/m,  1^T y1^j = 1^T (Rhat1^j + Q t) / n,
//   y3^l = (R3^l + t)/n.
// The global scalars are rebuilt by one wave from the reduce blocks'
// partials in a fixed order, so solve blocks need no communication.
//   kind 0, row block b: wave w writes beta of slabs 4(spw b + q) + w,
//           q < spw (F1 slabs j first, then F2 slabs k) and each slab's
//           (sum alpha, sum beta);
//   kind 1, tile (jt, kt): y1 on a 32 x 32 tile of (j, k), written as
//           alpha of F1^(j) (row j) and, transposed through LDS, as
//           -alpha of F2^(k) (row k).
// FROM_R = 1 is the entry point that solves for a given R (the reduce side
// then stores 1^T R1^j and sum_j R1[j][k] + PR3[k], and R1 itself).
// ---------------------------------------------------------------------------
struct SolveScalars {
  double sa, sp, u, sq, tlast;
};

template <int FROM_R>
__device__ inline double b1_of(const PairGeo& G, const double* vec, const double* ab, int j) {
  if (FROM_R) return vec[vec_b1(G) + j];
  return -(vec[vec_tot1(G) + j] - fam_cc(ab, G.f[0])) +
         (vec[vec_u2(G) + j] - (double)G.m * fam_cr(ab, G.f[1], j));
}

template <int FROM_R>
__device__ inline double Sp_of(const PairGeo& G, const double* vec, const double* ab, int k) {
  if (FROM_R) return vec[vec_Sp(G) + k];
  return -(vec[vec_u1(G) + k] - (double)G.n * fam_cr(ab, G.f[0], k)) +
         (vec[vec_tot2(G) + k] - fam_cc(ab, G.f[1])) + vec[vec_PR3(G) + k];
}

template <int FROM_R>
__device__ inline SolveScalars solve_scalars(const PairGeo& G, const double* vec, const double* ab,
                                             int lane) {
  const int m = G.m, n = G.n;
  const double dm = (double)m, dn = (double)n;
  const double* sp_ = vec + vec_spart(G);
  double sa = 0.0, sp = 0.0, up = 0.0;
  for (int b = lane; b < G.nblk + G.ns1; b += 64) {
    sa += sp_[4 * (int64_t)b];
    sp += sp_[4 * (int64_t)b + 1];
    up += sp_[4 * (int64_t)b + 2];
  }
  sa = wave_sum(sa);
  sp = wave_sum(sp);
  up = wave_sum(up);
  const double sdinv = (dm - 1.0) / dm + 1.0 / (dm + 1.0);
  SolveScalars S;
  S.sa = sa;
  S.sp = sp;
  S.u = up - (sa / dm) * sdinv;  // 1^T D^{-1} S
  const double Sl = Sp_of<FROM_R>(G, vec, ab, m - 1) - sa / dm;
  S.tlast = Sl / (dm + 1.0) + dm * (dm + 1.0) * S.u / (dm + 1.0);
  const double tsum = S.u * (1.0 + dm * (dm + 1.0) * sdinv);
  S.sq = tsum - S.tlast / dn;  // 1^T Q t
  return S;
}

// Inputs of a solve block that do not depend on the solve scalars, read
// before wave 0 has rebuilt them: for the first beta slab of a wave, the
// slab's scalar term without the scalar parts (F1: b1_j - a_j, so that
// rs_j = base + sp / n + 1^T Q t; F2: Sp_k, so that t_k = (base - sa / m) d_k
// + m (m+1) u d_k) and the lane's first two R2 / R3^T entries.
struct BetaPre {
  double base;
  double r0, r1;
};

template <int FROM_R>
__device__ __forceinline__ BetaPre beta_prefetch(const PairGeo& G, int slab, const double* arr,
                                        const double* vec, const double* ab, int lane) {
  BetaPre P{0.0, 0.0, 0.0};
  const int m = G.m, n = G.n;
  if (slab < n) {
    P.base = b1_of<FROM_R>(G, vec, ab, slab) - vec[vec_a(G) + slab];
    const double* R2 = arr + arr_R2(G) + (int64_t)slab * m;
    if (lane < m) P.r0 = R2[lane];
    if (lane + 64 < m) P.r1 = R2[lane + 64];
  } else if (slab < n + m) {
    const int k = slab - n;
    P.base = Sp_of<FROM_R>(G, vec, ab, k);
    const double* R3T = arr + arr_R3T(G) + (int64_t)k * n;
    if (lane < n) P.r0 = R3T[lane];
    if (lane + 64 < n) P.r1 = R3T[lane + 64];
  }
  return P;
}

// beta of one slab, and the slab's (sum alpha, sum beta): sum_k y1[j][k] =
// rs_j / n and sum_j y1[j][k] = t[k] in closed form.
template <int FROM_R>
__device__ __forceinline__ void solve_beta(const PairGeo& G, int slab, const double* arr,
                                           double* ab, const SolveScalars& S, int lane,
                                           const BetaPre P) {
  const int m = G.m, n = G.n;
  const double dm = (double)m, dn = (double)n;
  if (slab < n) {  // F1^(j): beta = y2[j][.]
    const int j = slab;
    const double* R2 = arr + arr_R2(G);
    const FamGeo F = G.f[0];
    double* be = ab + F.aboff + (int64_t)j * 2 * m + m;
    const double rsj = P.base + S.sp / dn + S.sq;
    double sb = 0.0;
    for (int i = lane, it = 0; i < m; i += 64, ++it) {
      const double r = it == 0 ? P.r0 : (it == 1 ? P.r1 : R2[(int64_t)j * m + i]);
      const double v = (r - rsj / dn) / dm;
      be[i] = v;
      sb += v;
    }
    sb = wave_sum(sb);
    if (lane == 0) {
      ab[F.sumoff + 2 * (int64_t)j] = rsj / dn;
      ab[F.sumoff + 2 * (int64_t)j + 1] = sb;
    }
  } else if (slab < n + m) {  // F2^(k): beta = y3[.][k]
    const int k = slab - n;
    const double* R3T = arr + arr_R3T(G);
    const FamGeo F = G.f[1];
    double* be = ab + F.aboff + (int64_t)k * 2 * n + n;
    const double d = dinv(m, k);
    const double tk = (P.base - S.sa / dm) * d + dm * (dm + 1.0) * S.u * d;
    double sb = 0.0;
    for (int l = lane, it = 0; l < n; l += 64, ++it) {
      const double r = it == 0 ? P.r0 : (it == 1 ? P.r1 : R3T[(int64_t)k * n + l]);
      const double v = (k == m - 1 && l == n - 1) ? 0.0 : (r + tk) / dn;
      be[l] = v;
      sb += v;
    }
    sb = wave_sum(sb);
    if (lane == 0) {
      ab[F.sumoff + 2 * (int64_t)k] = -tk;
      ab[F.sumoff + 2 * (int64_t)k + 1] = sb;
    }
  }
}

// y1 on a 32 x 32 tile of (j, k), in three parts around the decision:
//   tile_stage (waves 1-3, before it): R1 (or the F1 / F2 row sums) into LDS;
//   tile_pre / tile_scalars (wave 0, its lanes 0-31 for rows j and 32-63 for
//     columns k): the S-free row / column terms, loaded before the decision
//     and completed with the solve scalars after it;
//   solve_alpha_tile (every thread, after the barrier): y1, written as alpha
//     of F1^(j) (row j) and, transposed through LDS, as -alpha of F2^(k).
struct TileLds {
  double T1[32][33], T2[32][33];  // T1 holds R1 (or rs1) and then, in place, y1
  double rs[32], a[32], cn[32], qt[32], p3[32], cm[32];
};

struct TilePre {
  double base, x, y;  // rows: b1_j - a_j, a_j, C_n(j); columns: Sp_k, PR3_k, C_m(k)
};

template <int FROM_R>
__device__ __forceinline__ void tile_stage(const PairGeo& G, int tile, const double* rowsum,
                                  const double* arr, TileLds& L, int t0, int tstep) {
  const int m = G.m, n = G.n;
  const int j0 = 32 * (tile % G.ntj), k0 = 32 * (tile / G.ntj);
  const double* rs1 = rowsum + G.f[0].rsoff;  // [n][m]
  const double* rs2 = rowsum + G.f[1].rsoff;  // [m][n]
  const double* R1 = arr + arr_R1(G);
  for (int e = t0; e < 1024; e += tstep) {
    const int r = e >> 5, c = e & 31;
    const int j = j0 + r, k = k0 + c;        // T1[r][c] = (j, k)
    L.T1[r][c] = (j < n && k < m) ? (FROM_R ? R1[(int64_t)j * m + k] : rs1[(int64_t)j * m + k]) : 0.0;
    if (!FROM_R) {
      const int k2 = k0 + r, j2 = j0 + c;    // T2[r][c] = rs2[k2][j2]
      L.T2[r][c] = (k2 < m && j2 < n) ? rs2[(int64_t)k2 * n + j2] : 0.0;
    }
  }
}

template <int FROM_R>
__device__ __forceinline__ TilePre tile_pre(const PairGeo& G, int tile, const double* vec,
                                   const double* ab, int t) {
  TilePre P{0.0, 0.0, 0.0};
  const int j0 = 32 * (tile % G.ntj), k0 = 32 * (tile / G.ntj);
  if (t < 32) {
    const int j = j0 + t;
    if (j < G.n) {
      P.x = vec[vec_a(G) + j];
      P.base = b1_of<FROM_R>(G, vec, ab, j) - P.x;
      P.y = fam_cr(ab, G.f[1], j);
    }
  } else {
    const int k = k0 + t - 32;
    if (k < G.m) {
      P.base = Sp_of<FROM_R>(G, vec, ab, k);
      P.x = vec[vec_PR3(G) + k];
      P.y = fam_cr(ab, G.f[0], k);
    }
  }
  return P;
}

__device__ __forceinline__ void tile_scalars(const PairGeo& G, int tile, const TilePre P,
                                    const SolveScalars& S, TileLds& L, int t) {
  const double dm = (double)G.m, dn = (double)G.n;
  const int j0 = 32 * (tile % G.ntj), k0 = 32 * (tile / G.ntj);
  if (t < 32) {
    if (j0 + t < G.n) {
      L.rs[t] = P.base + S.sp / dn + S.sq;
      L.a[t] = P.x;
      L.cn[t] = P.y;
    }
  } else {
    const int kk = t - 32, k = k0 + kk;
    if (k < G.m) {
      const double d = dinv(G.m, k);
      const double tk = (P.base - S.sa / dm) * d + dm * (dm + 1.0) * S.u * d;
      L.qt[kk] = (k == G.m - 1) ? tk - tk / dn : tk;
      L.p3[kk] = P.x;
      L.cm[kk] = P.y;
    }
  }
}

template <int FROM_R>
__device__ __forceinline__ void solve_alpha_tile(const PairGeo& G, int tile, double* ab,
                                                 TileLds& L) {
  const int m = G.m, n = G.n;
  const double dm = (double)m, dn = (double)n;
  const int j0 = 32 * (tile % G.ntj), k0 = 32 * (tile / G.ntj);
  const int t = threadIdx.x;
  const FamGeo F1 = G.f[0], F2 = G.f[1];
  for (int e = t; e < 1024; e += kWG) {
    const int jj = e >> 5, kk = e & 31;
    const int j = j0 + jj, k = k0 + kk;
    if (j < n && k < m) {
      const double r1 =
          FROM_R ? L.T1[jj][kk] : -(L.T1[jj][kk] - L.cm[kk]) + (L.T2[kk][jj] - L.cn[jj]);
      const double rh = r1 - L.a[jj] / dm + L.p3[kk] / dn;
      const double y = (rh + L.qt[kk] + L.rs[jj] / dn) / (dm + dn);
      ab[F1.aboff + (int64_t)j * 2 * m + k] = y;
      L.T1[jj][kk] = y;  // (this thread alone read T1[jj][kk] above)
    }
  }
  __syncthreads();
  for (int e = t; e < 1024; e += kWG) {
    const int kk = e >> 5, jj = e & 31;
    const int j = j0 + jj, k = k0 + kk;
    if (j < n && k < m) ab[F2.aboff + (int64_t)k * 2 * n + j] = -L.T1[jj][kk];
  }
}

// PRE = 1 (the default): the loads that need no decision go out before it
// (wasted only on the pass that stops the pair), waves 1-3 staging the tile
// while wave 0 decides.  PRE = 0 issues them after it (fewer registers held
// across the decision: 69 against 79 VGPRs).  Same arithmetic.
// One solve block's work (the body of k_pair_solve, also the solve role of
// k_pair_fused).
template <int FROM_R, int PRE>
__device__ __forceinline__ void solve_block(const PBlock pbk, const PairGeo* __restrict__ geo,
                                            const PairCtl* __restrict__ ctl,
                                            PairCtl* __restrict__ ctl_next,
                                            const double* __restrict__ rowsum,
                                            const double* __restrict__ arr,
                                            const double* __restrict__ vec,
                                            double* __restrict__ ab) {
  __shared__ PairCtl s_nx;
  __shared__ SolveScalars s_S;
  __shared__ int s_solve;
  __shared__ TileLds s_tile;
  const bool head = (pbk.kind == 0 && pbk.blk == 0 && threadIdx.x == 0);
  if (!FROM_R) {
    const PairCtl* cp = ctl + pbk.pair;
    if (cp->status != ST_RUNNING || cp->mode == MODE_IDLE) {
      if (head) ctl_next[pbk.pair] = *cp;
      return;
    }
  }
  const PairGeo G = geo[pbk.pair];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // (kind 1, wave 0: holds the tile's row / column terms as base, r0, r1)
  BetaPre bp{0.0, 0.0, 0.0};
  if constexpr (PRE) {
    if (pbk.kind == 0) {
      bp = beta_prefetch<FROM_R>(G, 4 * G.spw * pbk.blk + wave, arr, vec, ab, lane);
    } else if (wave == 0) {
      const TilePre tp = tile_pre<FROM_R>(G, pbk.blk, vec, ab, lane);
      bp = BetaPre{tp.base, tp.x, tp.y};
    } else {
      tile_stage<FROM_R>(G, pbk.blk, rowsum, arr, s_tile, threadIdx.x - 64, kWG - 64);
    }
  }
  if (wave == 0) {  // wave 0 decides and rebuilds the solve scalars
    bool solve = true;
    PairCtl nx;
    if (!FROM_R) {
      const PairCtl c = ctl[pbk.pair];
      double acc[kNKP];
      if (c.mode == MODE_CHECK) reduce_kpart(G, vec, lane, acc);
      decide(G, c, acc, nx, solve);
    }
    SolveScalars S;
    if (solve) {
      S = solve_scalars<FROM_R>(G, vec, ab, lane);
      if (PRE && pbk.kind != 0)
        tile_scalars(G, pbk.blk, TilePre{bp.base, bp.r0, bp.r1}, S, s_tile, lane);
    }
    if (lane == 0) {
      if (!FROM_R) s_nx = nx;
      s_solve = solve ? 1 : 0;
      if (solve) s_S = S;
    }
  }
  __syncthreads();
  if (s_solve) {
    if (pbk.kind == 0) {
      for (int q = 0; q < G.spw; ++q) {  // slabs 4 (spw b + q) + w
        const int slab = 4 * (G.spw * pbk.blk + q) + wave;
        const BetaPre P =
            (PRE && q == 0) ? bp : beta_prefetch<FROM_R>(G, slab, arr, vec, ab, lane);
        solve_beta<FROM_R>(G, slab, arr, ab, s_S, lane, P);
      }
    } else {
      if constexpr (!PRE) {
        if (wave == 0) {
          const TilePre tp = tile_pre<FROM_R>(G, pbk.blk, vec, ab, lane);
          tile_scalars(G, pbk.blk, tp, s_S, s_tile, lane);
        }
        tile_stage<FROM_R>(G, pbk.blk, rowsum, arr, s_tile, threadIdx.x, kWG);
        __syncthreads();
      }
      solve_alpha_tile<FROM_R>(G, pbk.blk, ab, s_tile);
    }
  }
  if (!FROM_R && head) ctl_next[pbk.pair] = s_nx;
}

template <int FROM_R, int PRE>
__global__ __launch_bounds__(kWG) void k_pair_solve(const PBlock* __restrict__ sblocks,
                                                    const PairGeo* __restrict__ geo,
                                                    const PairCtl* __restrict__ ctl,
                                                    PairCtl* __restrict__ ctl_next,
                                                    const double* __restrict__ rowsum,
                                                    const double* __restrict__ arr,
                                                    const double* __restrict__ vec,
                                                    double* __restrict__ ab) {
  solve_block<FROM_R, PRE>(sblocks[blockIdx.x], geo, ctl, ctl_next, rowsum, arr, vec, ab);
}

// ---------------------------------------------------------------------------
// Reduce and solve in one launch (HOT_FUSE_PAIR=1): workgroups [0, nblocks)
// take the reduce blocks, the rest the solve blocks.  A reduce workgroup
// publishes its outputs (device-scope release) and counts itself in its
// pair's counter; a solve workgroup waits until its pair's count is complete
// (device-scope acquire), then solves.  Every reduce workgroup has a lower
// index than every solve workgroup, and workgroups of one launch are
// dispatched in index order, so all reduce workgroups are dispatched before
// any solve workgroup that could occupy their place, and the waits end.  The
// wait is bounded all the same: past kFuseSpin polls the workgroup marks the
// pair in `lost` and solves anyway; the finalize pass turns the mark into a
// device error for that problem.  The last solve workgroup of a pair clears
// its counters for the launch two iterations on (counters alternate with the
// control-block parity).
// ---------------------------------------------------------------------------
constexpr unsigned kFuseSpin = 1u << 20;

template <int PRE>
__global__ __launch_bounds__(kWG) void k_pair_fused(
    const PBlock* __restrict__ blocks, int nblocks, const PBlock* __restrict__ sblocks,
    const PairGeo* __restrict__ geo, const PairCtl* __restrict__ ctl,
    PairCtl* __restrict__ ctl_next, const double* __restrict__ rowsum,
    const double* __restrict__ colpart, const double* __restrict__ rowsum_prev,
    const double* __restrict__ colpart_prev, const double* __restrict__ kitem,
    double* __restrict__ ab, double* __restrict__ abY, double* __restrict__ arr,
    double* __restrict__ vec, unsigned long long* __restrict__ bytes_ctr, int elem,
    unsigned* __restrict__ sync, unsigned* __restrict__ lost) {
  const bool red = (int)blockIdx.x < nblocks;
  const PBlock pbk = red ? blocks[blockIdx.x] : sblocks[blockIdx.x - nblocks];
  const PairCtl* cp = ctl + pbk.pair;
  const bool live = cp->status == ST_RUNNING && cp->mode != MODE_IDLE;
  unsigned* cnt = sync + 2 * (int64_t)pbk.pair;  // (reduce count, solve count)
  if (red) {
    if (!live) return;
    reduce_block(pbk, geo, ctl, rowsum, colpart, rowsum_prev, colpart_prev, kitem, ab, abY, arr,
                 vec, bytes_ctr, elem);
    __syncthreads();  // every wave's stores are done
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  if (live && threadIdx.x == 0) {
    const unsigned want = (unsigned)reduce_blocks_of(geo[pbk.pair]);
    unsigned polls = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want &&
           ++polls < kFuseSpin)
      __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (polls >= kFuseSpin)
      __hip_atomic_fetch_or(lost + pbk.pair, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  solve_block<0, PRE>(pbk, geo, ctl, ctl_next, rowsum, arr, vec, ab);
  if (live) {
    __syncthreads();
    if (threadIdx.x == 0 &&
        __hip_atomic_fetch_add(cnt + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
            (unsigned)solve_blocks_of(geo[pbk.pair]) - 1u) {
      // every solve workgroup of the pair is past its wait
      __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(cnt + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// Finalize (once per solve, after the last check): the feasibility error of
// the experiments, max(||min(x_bar, 0)|| / (1 + ||x_bar||), res_primal), of
// the final iterate x_bar = sigma (s - g).  A reporting metric only, so it is
// kept out of the slab pass (an eighth check accumulator there cost the
// streaming kernel 20 VGPRs and a wave per SIMD).  One workgroup per slab
// item writes the item's (||x_bar||^2, ||x_bar^-||^2) into its partial slots;
// one workgroup per problem adds them in a fixed order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kWG) void k_feas_items(const SlabItem* __restrict__ items,
                                                    const PairGeo* __restrict__ geo,
                                                    const PairCtl* __restrict__ ctl,
                                                    const T* __restrict__ sb0,
                                                    const T* __restrict__ sb1,
                                                    const T* __restrict__ sb2,
                                                    const double* __restrict__ ab,
                                                    double* __restrict__ kitem) {
  __shared__ double red[4];
  const SlabItem itm = items[blockIdx.x];
  const PairCtl* cp = ctl + itm.pair;
  const FamGeo F = geo[itm.pair].f[itm.fam];
  const int L = F.L;
  const T* s = pick<const T>(sb0, sb1, sb2, cp->src) + F.soff + (int64_t)itm.slab * L * F.P;
  const double* alpha = ab + F.aboff + (int64_t)itm.slab * 2 * L;
  const double* beta = alpha + L;
  const double* X = fam_x(ab, F);
  const double sigma = cp->sigma;
  const int r0 = itm.chunk * F.rpc, r1 = min(L, r0 + F.rpc);
  const int64_t cnt = (int64_t)(r1 - r0) * L;
  double xx = 0.0, neg = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += kWG) {
    const int p = r0 + (int)(e / L), q = (int)(e % L);
    const double d = X[p] - X[q];
    const double g = d * d - (alpha[p] + beta[q]);
    const double xb = sigma * ((double)s[(int64_t)p * F.P + q] - g);
    const double xn = fmin(xb, 0.0);
    xx += xb * xb;
    neg += xn * xn;
  }
  xx = block_sum(xx, red);
  neg = block_sum(neg, red);
  if (threadIdx.x == 0) {
    kitem[(int64_t)itm.kslot * kKI + KI_DX] = xx;
    kitem[(int64_t)itm.kslot * kKI + KI_NEG] = neg;
  }
}

__global__ __launch_bounds__(kWG) void k_feas_pairs(const PairGeo* __restrict__ geo,
                                                    PairCtl* __restrict__ ctl,
                                                    const double* __restrict__ kitem,
                                                    const unsigned* __restrict__ lost) {
  __shared__ double red[4];
  const PairGeo G = geo[blockIdx.x];
  double xx = 0.0, neg = 0.0;
  for (int it = G.item0 + (int)threadIdx.x; it < G.item0 + G.nitem; it += kWG) {
    xx += kitem[(int64_t)it * kKI + KI_DX];
    neg += kitem[(int64_t)it * kKI + KI_NEG];
  }
  xx = block_sum(xx, red);
  neg = block_sum(neg, red);
  if (threadIdx.x == 0) {
    PairCtl* c = ctl + blockIdx.x;
    c->feaserr = fmax(sqrt(neg) / (1.0 + sqrt(xx)), c->res_p);
    if (lost && lost[blockIdx.x]) {  // a fused reduce + solve wait ran out
      c->status = ST_SYNC_LOST;
      c->mode = MODE_IDLE;
    }
  }
}

// ---------------------------------------------------------------------------
// Setup and export helpers.
// ---------------------------------------------------------------------------

// Input check, one block per histogram: min, total, non-finite count, sum of
// squares and last entry (the last target entry is not a row of b).
__global__ __launch_bounds__(kWG) void k_hist_stats_multi(const double* const* __restrict__ ptrs,
                                                          const int64_t* __restrict__ lens,
                                                          double* __restrict__ out) {
  __shared__ double red[4];
  __shared__ double mred[4];
  const double* mu = ptrs[blockIdx.x];
  const int64_t len = lens[blockIdx.x];
  double mn = INFINITY, sum = 0.0, bad = 0.0, sq = 0.0;
  for (int64_t q = threadIdx.x; q < len; q += kWG) {
    const double v = mu[q];
    if (!isfinite(v)) {
      bad += 1.0;
    } else {
      mn = fmin(mn, v);
      sum += v;
      sq += v * v;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) mn = fmin(mn, __shfl_xor(mn, off, 64));
  if ((threadIdx.x & 63) == 0) mred[threadIdx.x >> 6] = mn;
  sum = block_sum(sum, red);
  bad = block_sum(bad, red);
  sq = block_sum(sq, red);
  if (threadIdx.x == 0) {
    double* o = out + (int64_t)blockIdx.x * 8;
    o[0] = fmin(fmin(mred[0], mred[1]), fmin(mred[2], mred[3]));
    o[1] = sum;
    o[2] = bad;
    o[3] = sq;
    o[4] = len > 0 ? mu[len - 1] : 0.0;
  }
}

// Zero fill: 16-byte stores over the aligned body, 4-byte stores for a tail
// (every buffer is 256-byte aligned and a multiple of 4 bytes long).
__global__ void k_zero(uint4* __restrict__ p, int64_t n16, uint32_t* __restrict__ tail,
                       int64_t ntail) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t q = t0; q < n16; q += stride) p[q] = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t q = t0; q < ntail; q += stride) tail[q] = 0u;
}

// FP32 state widened to FP64 (exact).
__global__ void k_widen(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (double)in[e];
}

// mu1T[j][i] = mu1[i][j], mu2[k][l] copied.
__global__ void k_setup_mu(const double* __restrict__ mu1, const double* __restrict__ mu2,
                           int m, int n, double* __restrict__ mu1T, double* __restrict__ mu2c) {
  const int64_t M = (int64_t)m * n;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < M;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(q / n), j = (int)(q % n);
    mu1T[(int64_t)j * m + i] = mu1[q];
    mu2c[q] = mu2[q];
  }
}

// Export the final iterate of one pair in the paper's ordering.
template <typename T>
__global__ void k_export(const PairGeo* __restrict__ geo, const PairCtl* __restrict__ ctl, int pair,
                         const T* __restrict__ sb0, const T* __restrict__ sb1,
                         const T* __restrict__ sb2, const double* __restrict__ ab,
                         double* __restrict__ xbar, double* __restrict__ zbar,
                         double* __restrict__ sout, double* __restrict__ s0out) {
  const PairGeo G = geo[pair];
  const PairCtl c = ctl[pair];
  const int m = G.m, n = G.n;
  const int64_t N1 = (int64_t)m * m * n, N = N1 + (int64_t)m * n * n;
  const T* s = pick<const T>(sb0, sb1, sb2, c.src);
  // the Halpern anchor of the epoch: zero before the first restart
  const T* s0 = c.anc >= 0 ? pick<const T>(sb0, sb1, sb2, c.anc) : nullptr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    int fam, slab, p, q, L;
    if (e < N1) {  // x1 index (j*m + k)*m + i
      const int i = (int)(e % m);
      const int64_t r = e / m;
      const int k = (int)(r % m), j = (int)(r / m);
      fam = 0; slab = j; p = k; q = i; L = m;
    } else {       // x2 index (l*n + j)*m + k
      const int64_t e2 = e - N1;
      const int k = (int)(e2 % m);
      const int64_t r = e2 / m;
      const int j = (int)(r % n), l = (int)(r / n);
      fam = 1; slab = k; p = j; q = l; L = n;
    }
    const FamGeo F = G.f[fam];
    const int64_t at = F.soff + ((int64_t)slab * L + p) * F.P + q;
    const double sv = (double)s[at];
    if (s0out) s0out[e] = s0 ? (double)s0[at] : 0.0;
    const double* al = ab + F.aboff + (int64_t)slab * 2 * L;
    const double* X = fam_x(ab, F);
    const double d = X[p] - X[q];
    const double g = d * d - al[p] - al[L + q];
    if (xbar) xbar[e] = c.sigma * (sv - g);
    if (zbar) zbar[e] = fmax(0.0, 2.0 * g - sv);
    if (sout) sout[e] = sv;
  }
}

__global__ void k_export_y(const PairGeo* __restrict__ geo, int pair, const double* __restrict__ ab,
                           double* __restrict__ y) {
  const PairGeo G = geo[pair];
  const int m = G.m, n = G.n;
  const int64_t M = (int64_t)m * n;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < 3 * M - 1;
       q += (int64_t)gridDim.x * blockDim.x) {
    double v;
    if (q < M) {            // y1[j][k] = alpha of F1^(j) at k
      const int j = (int)(q / m), k = (int)(q % m);
      v = ab[G.f[0].aboff + (int64_t)j * 2 * m + k];
    } else if (q < 2 * M) { // y2[j][i] = beta of F1^(j) at i
      const int64_t r = q - M;
      const int j = (int)(r / m), i = (int)(r % m);
      v = ab[G.f[0].aboff + (int64_t)j * 2 * m + m + i];
    } else {                // y3[l][k] = beta of F2^(k) at l
      const int64_t r = q - 2 * M;
      const int l = (int)(r / m), k = (int)(r % m);
      v = ab[G.f[1].aboff + (int64_t)k * 2 * n + n + l];
    }
    y[q] = v;
  }
}

// R in the paper's order -> R1[j][k], R2[j][i], R3T[k][l] (for hot_aat_solve).
__global__ void k_scatter_R(const PairGeo* __restrict__ geo, int pair, const double* __restrict__ R,
                            double* __restrict__ arr) {
  const PairGeo G = geo[pair];
  const int m = G.m, n = G.n;
  const int64_t M = (int64_t)m * n;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < 3 * M;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (q < 2 * M) {
      arr[(q < M ? arr_R1(G) : arr_R2(G)) + (q % M)] = R[q];
    } else {
      const int64_t r = q - 2 * M;
      const int l = (int)(r / m), k = (int)(r % m);
      arr[arr_R3T(G) + (int64_t)k * n + l] = (r == M - 1) ? 0.0 : R[q];
    }
  }
}

// Totals of the solve from stored R arrays (entry point with R given): the
// quantities k_pair_reduce produces from slab sums, taken from R directly.
__global__ __launch_bounds__(kWG) void k_pair_sums_from_R(const PBlock* __restrict__ blocks,
                                                          const PairGeo* __restrict__ geo,
                                                          const double* __restrict__ arr,
                                                          double* __restrict__ vec) {
  __shared__ double wred[4][kKP];
  __shared__ double blk_red[4];
  const PBlock pbk = blocks[blockIdx.x];
  const PairGeo G = geo[pbk.pair];
  const int m = G.m, n = G.n, b = pbk.blk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (pbk.kind == 1 || pbk.kind == 2) {  // strip slots carry no partial on this path
    if (pbk.kind == 1 && threadIdx.x < 4) vec[vec_spart(G) + 4 * (int64_t)(G.nblk + b) + threadIdx.x] = 0.0;
    return;
  }
  const bool f1 = pbk.kind == 0;
  const double* R1 = arr + arr_R1(G);
  const double* R2 = arr + arr_R2(G);
  const double* R3T = arr + arr_R3T(G);
  // the reduce's block shapes: one wave per slab, or the block for a wide family
  const bool wide = (f1 ? G.f[0].wide : G.f[1].wide) != 0;
  const int nq = wide ? 1 : G.rq;
  const int nslot = f1 ? G.nb1 : G.nblk - G.nb1;
  for (int qd = 0; qd < nq; ++qd) {
    const int sq = nq * b + qd;  // slot within the family
    if (sq >= nslot) break;
    if (qd > 0) __syncthreads();  // the previous slot's wred has been read
    const int slot = f1 ? sq : G.nb1 + sq;
    const int r = wide ? sq : 4 * sq + wave;
    const int tid = wide ? (int)threadIdx.x : lane;
    const int nthr = wide ? kWG : 64;
    auto slab_sum = [&](double v) { return wide ? block_sum(v, blk_red) : wave_sum(v); };
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    if (f1 && r < n) {
      const int j = r;
      double s1 = 0.0, s2 = 0.0;
      for (int kk = tid; kk < m; kk += nthr) s1 += R1[(int64_t)j * m + kk];
      for (int i = tid; i < m; i += nthr) s2 += R2[(int64_t)j * m + i];
      s1 = slab_sum(s1);
      s2 = slab_sum(s2);
      if (tid == 0) {
        vec[vec_b1(G) + j] = s1;
        vec[vec_a(G) + j] = s2;
      }
      p0 = s2;
    } else if (!f1 && r < m) {
      const int k = r;
      double s3 = 0.0, c1 = 0.0;
      for (int l = tid; l < n; l += nthr) s3 += R3T[(int64_t)k * n + l];
      for (int jj = tid; jj < n; jj += nthr) c1 += R1[(int64_t)jj * m + k];
      s3 = slab_sum(s3);
      c1 = slab_sum(c1);
      if (tid == 0) {
        vec[vec_PR3(G) + k] = s3;
        vec[vec_Sp(G) + k] = c1 + s3;
      }
      p1 = s3;
      p2 = (c1 + s3) * dinv(m, k);
    }
    if (wide && wave != 0) p0 = p1 = p2 = 0.0;  // (every wave holds the slab totals)
    if (lane == 0) {
      wred[wave][0] = p0;
      wred[wave][1] = p1;
      wred[wave][2] = p2;
    }
    __syncthreads();
    if (threadIdx.x < 3)
      vec[vec_spart(G) + 4 * (int64_t)slot + threadIdx.x] = wave4(wred, threadIdx.x);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage inside the library).
// ---------------------------------------------------------------------------

template <int FROM_R>
static void launch_solve(const LaunchArgs& a, const PairCtl* ctl, PairCtl* ctl_next,
                         const double* rowsum, hipStream_t st) {
  if (a.solve_pre != 0)
    hipLaunchKernelGGL((k_pair_solve<FROM_R, 1>), dim3(a.nsblocks), dim3(kWG), 0, st, a.sblocks,
                       a.geo, ctl, ctl_next, rowsum, a.arr, a.vec, a.ab);
  else
    hipLaunchKernelGGL((k_pair_solve<FROM_R, 0>), dim3(a.nsblocks), dim3(kWG), 0, st, a.sblocks,
                       a.geo, ctl, ctl_next, rowsum, a.arr, a.vec, a.ab);
}

void launch_pair_kernels(const LaunchArgs& a, int par, hipStream_t st) {
  if (a.fuse_pair && a.sync[par]) {
    const dim3 grid(a.nblocks + a.nsblocks);
    if (a.solve_pre != 0)
      hipLaunchKernelGGL(k_pair_fused<1>, grid, dim3(kWG), 0, st, a.blocks, a.nblocks, a.sblocks,
                         a.geo, a.ctl[par], a.ctl[1 - par], a.rowsum[par], a.colpart[par],
                         a.rowsum[1 - par], a.colpart[1 - par], a.kitem, a.ab, a.abY, a.arr,
                         a.vec, a.bytes_ctr, a.fp32 ? 4 : 8, a.sync[par], a.lost);
    else
      hipLaunchKernelGGL(k_pair_fused<0>, grid, dim3(kWG), 0, st, a.blocks, a.nblocks, a.sblocks,
                         a.geo, a.ctl[par], a.ctl[1 - par], a.rowsum[par], a.colpart[par],
                         a.rowsum[1 - par], a.colpart[1 - par], a.kitem, a.ab, a.abY, a.arr,
                         a.vec, a.bytes_ctr, a.fp32 ? 4 : 8, a.sync[par], a.lost);
    return;
  }
  hipLaunchKernelGGL(k_pair_reduce, dim3(a.nblocks), dim3(kWG), 0, st, a.blocks, a.geo,
                     a.ctl[par], a.rowsum[par], a.colpart[par], a.rowsum[1 - par],
                     a.colpart[1 - par], a.kitem, a.ab, a.abY, a.arr, a.vec, a.bytes_ctr,
                     a.fp32 ? 4 : 8);
  launch_solve<0>(a, a.ctl[par], a.ctl[1 - par], (const double*)a.rowsum[par], st);
}

// One iteration: slab pass, pair reduce, pair solve (or the two in one
// launch).  Reads ctl[par], writes ctl[1-par].
void launch_iteration(const LaunchArgs& a, int par, hipStream_t st) {
  launch_slab_pass(a, par, st);
  launch_pair_kernels(a, par, st);
}

void launch_hist_stats_multi(const double* const* ptrs, const int64_t* lens, int count,
                             double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_hist_stats_multi, dim3(count), dim3(kWG), 0, st, ptrs, lens, out);
}

// Finalize every problem of a workspace (full launch tables, control blocks
// ctl[0], which hold the final state after whole graphs).
void launch_finalize(const LaunchArgs& a, const SlabItem* items_all, int nitems_all, int npairs,
                     hipStream_t st) {
  if (nitems_all < 1 || npairs < 1) return;
  if (a.fp32)
    hipLaunchKernelGGL(k_feas_items<float>, dim3(nitems_all), dim3(kWG), 0, st, items_all, a.geo,
                       a.ctl[0], (const float*)a.sb[0], (const float*)a.sb[1],
                       (const float*)a.sb[2], a.ab, a.kitem);
  else
    hipLaunchKernelGGL(k_feas_items<double>, dim3(nitems_all), dim3(kWG), 0, st, items_all,
                       a.geo, a.ctl[0], (const double*)a.sb[0], (const double*)a.sb[1],
                       (const double*)a.sb[2], a.ab, a.kitem);
  hipLaunchKernelGGL(k_feas_pairs, dim3(npairs), dim3(kWG), 0, st, a.geo, a.ctl[0], a.kitem,
                     a.lost);
}

void launch_widen(const void* in, void* out, int64_t n, hipStream_t st) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kWG - 1) / kWG, 65536));
  hipLaunchKernelGGL(k_widen, dim3(grid), dim3(kWG), 0, st, (const float*)in, (double*)out, n);
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (!p || bytes < 4) return;
  const int64_t n16 = (int64_t)(bytes / 16);
  const int64_t ntail = (int64_t)((bytes - 16 * (size_t)n16) / 4);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n16 + kWG - 1) / kWG, 8192));
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(kWG), 0, st, (uint4*)p, n16,
                     (uint32_t*)((char*)p + 16 * n16), ntail);
}

void launch_setup_mu(const double* mu1, const double* mu2, int m, int n, double* mu1T,
                     double* mu2c, hipStream_t st) {
  const int64_t M = (int64_t)m * n;
  const int grid = (int)std::min<int64_t>((M + kWG - 1) / kWG, 4096);
  hipLaunchKernelGGL(k_setup_mu, dim3(grid), dim3(kWG), 0, st, mu1, mu2, m, n, mu1T, mu2c);
}

void launch_export(const LaunchArgs& a, int par, int pair, int64_t N, double* xbar,
                   double* zbar, double* sout, hipStream_t st, double* s0out) {
  const int grid = (int)std::min<int64_t>((N + kWG - 1) / kWG, 65536);
  if (a.fp32)
    hipLaunchKernelGGL(k_export<float>, dim3(grid), dim3(kWG), 0, st, a.geo, a.ctl[par], pair,
                       (const float*)a.sb[0], (const float*)a.sb[1], (const float*)a.sb[2], a.ab,
                       xbar, zbar, sout, s0out);
  else
    hipLaunchKernelGGL(k_export<double>, dim3(grid), dim3(kWG), 0, st, a.geo, a.ctl[par], pair,
                       (const double*)a.sb[0], (const double*)a.sb[1], (const double*)a.sb[2],
                       a.ab, xbar, zbar, sout, s0out);
}

void launch_export_y(const LaunchArgs& a, int pair, int64_t M3, double* y, hipStream_t st) {
  const int grid = (int)std::min<int64_t>((M3 + kWG - 1) / kWG, 65536);
  hipLaunchKernelGGL(k_export_y, dim3(grid), dim3(kWG), 0, st, a.geo, pair, a.ab, y);
}

void launch_aat_solve(const LaunchArgs& a, int pair, int64_t M, const double* R,
                      hipStream_t st) {
  const int grid = (int)std::min<int64_t>((3 * M + kWG - 1) / kWG, 65536);
  hipLaunchKernelGGL(k_scatter_R, dim3(grid), dim3(kWG), 0, st, a.geo, pair, R, a.arr);
  hipLaunchKernelGGL(k_pair_sums_from_R, dim3(a.nblocks), dim3(kWG), 0, st, a.blocks, a.geo,
                     a.arr, a.vec);
  launch_solve<1>(a, nullptr, nullptr, nullptr, st);
}

}  // namespace hot

// HIP kernels of the HOT iteration (arXiv 2408.00598, Algorithm 2) for gfx950.
//
// One iteration is three launches:
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
#include "hot_internal.h"
#include "hot_runtime.h"

#include <algorithm>

namespace hot {

template <typename T>
struct VecT;
template <>
struct VecT<float> {
  static constexpr int W = 4;
  typedef float4 type;
};
template <>
struct VecT<double> {
  static constexpr int W = 2;
  typedef double2 type;
};

__device__ inline float vget(const float4& v, int e) {
  return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}
__device__ inline double vget(const double2& v, int e) { return e == 0 ? v.x : v.y; }
__device__ inline void vset(float4& v, int e, float x) {
  if (e == 0) v.x = x; else if (e == 1) v.y = x; else if (e == 2) v.z = x; else v.w = x;
}
__device__ inline void vset(double2& v, int e, double x) {
  if (e == 0) v.x = x; else v.y = x;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 256 threads of a block, fixed order; every thread gets it.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T>
__device__ inline T* pick(T* b0, T* b1, T* b2, int i) {
  return i == 0 ? b0 : (i == 1 ? b1 : b2);
}

// ---------------------------------------------------------------------------
// Slab pass.  One workgroup per (slab, row chunk).  A row of the slab is
// covered by LR = 2^lrs lanes, each holding vpl 16-byte vectors of the row;
// a wave covers 64/LR rows per step, the four waves interleave.  Column
// sums stay in FP64 registers for the whole chunk; row sums are finished
// with a shuffle tree across the LR lanes of the row.
// ---------------------------------------------------------------------------
template <typename T, int MAXVPL>
__global__ __launch_bounds__(kWG) void k_slab_pass(
    const SlabItem* __restrict__ items, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, T* __restrict__ sb0, T* __restrict__ sb1,
    T* __restrict__ sb2, const double* __restrict__ ab, double* __restrict__ rowsum,
    double* __restrict__ colpart, double* __restrict__ kitem) {
  constexpr int W = VecT<T>::W;
  typedef typename VecT<T>::type VT;
  __shared__ double lds_col[4 * 64 * MAXVPL * W];
  __shared__ double red[4];

  const SlabItem itm = items[blockIdx.x];
  const PairCtl* cp = ctl + itm.pair;
  const int status = cp->status;
  const int mode = cp->mode;
  if (status != ST_RUNNING) return;
  if (mode != MODE_NORMAL && mode != MODE_CHECK && mode != MODE_RESTART) return;
  const FamGeo F = geo[itm.pair].f[itm.fam];
  const int L = F.L, P = F.P;
  const int r0 = itm.chunk * F.rpc;
  const int r1 = min(L, r0 + F.rpc);
  const int64_t soff = F.soff + (int64_t)itm.slab * L * P;
  const int src_i = cp->src, anc_i = cp->anc;
  const int dst_i = (mode == MODE_RESTART) ? 2 : cp->dst;
  const T* __restrict__ src = pick<T>(sb0, sb1, sb2, src_i) + soff;
  T* __restrict__ dst = pick<T>(sb0, sb1, sb2, dst_i) + soff;
  // anchor: -1 zero, == src the same values as s (first update of an epoch)
  const bool anc_zero = (anc_i < 0) || (mode == MODE_RESTART);
  const bool anc_same = !anc_zero && (anc_i == src_i);
  const T* __restrict__ anc = (anc_zero || anc_same) ? src : pick<T>(sb0, sb1, sb2, anc_i) + soff;
  const double lam = cp->lam, oml = 1.0 - cp->lam, sigma = cp->sigma;
  const double* __restrict__ alpha = ab + F.aboff + (int64_t)itm.slab * 2 * L;
  const double* __restrict__ beta = alpha + L;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lrs = F.lrs, LR = 1 << lrs;
  const int slot = lane >> lrs, lin = lane & (LR - 1);
  const int rpw = 64 >> lrs;
  const int vpl = F.vpl;

  double bq[MAXVPL][W], colacc[MAXVPL][W];
#pragma unroll
  for (int v = 0; v < MAXVPL; ++v)
#pragma unroll
    for (int e = 0; e < W; ++e) {
      const int q = ((lin + (v << lrs)) * W) + e;
      bq[v][e] = (v < vpl && q < L) ? beta[q] : 0.0;
      colacc[v][e] = 0.0;
    }
  double kd = 0, kc = 0, kx = 0, kz = 0, kcx = 0, kfp = 0;

  for (int pb = r0 + wave * rpw; pb < r1; pb += 4 * rpw) {
    const int p = pb + slot;
    const bool rv = p < r1;
    const double ap = rv ? alpha[p] : 0.0;
    double rowacc = 0.0;
    VT xs[MAXVPL], xa[MAXVPL];
#pragma unroll
    for (int v = 0; v < MAXVPL; ++v) {
      const int q0 = (lin + (v << lrs)) * W;
      if (v < vpl && rv && q0 < L) {
        xs[v] = *reinterpret_cast<const VT*>(src + (int64_t)p * P + q0);
        if (!anc_zero && !anc_same) xa[v] = *reinterpret_cast<const VT*>(anc + (int64_t)p * P + q0);
      }
    }
#pragma unroll
    for (int v = 0; v < MAXVPL; ++v) {
      const int q0 = (lin + (v << lrs)) * W;
      if (v < vpl && rv && q0 < L) {
        VT out;
#pragma unroll
        for (int e = 0; e < W; ++e) {
          const int q = q0 + e;
          T st = (T)0;
          if (q < L) {
            const double s = (double)vget(xs[v], e);
            const double d = (double)(p - q);
            const double g = d * d - ap - bq[v][e];
            double o;
            if (mode == MODE_RESTART) {
              o = fmax(s - g, g);
            } else {
              const double sh = fabs(s - 2.0 * g);
              const double a = anc_zero ? 0.0 : (anc_same ? s : (double)vget(xa[v], e));
              o = lam * a + oml * sh;
              if (mode == MODE_CHECK) {
                const double xb = sigma * (s - g);
                const double zb = fmax(0.0, 2.0 * g - s);
                const double dr = zb - g;
                const double mn = fmin(xb, zb);
                const double fr = s - sh;
                kd += dr * dr;
                kc += mn * mn;
                kx += xb * xb;
                kz += zb * zb;
                kcx += d * d * xb;
                kfp += fr * fr;
              }
            }
            st = (T)o;
            const double sd = (double)st;
            rowacc += sd;
            colacc[v][e] += sd;
          }
          vset(out, e, st);
        }
        *reinterpret_cast<VT*>(dst + (int64_t)p * P + q0) = out;
      }
    }
    // row sum across the LR lanes of this row
    for (int off = 1; off < LR; off <<= 1) rowacc += __shfl_xor(rowacc, off, 64);
    if (rv && lin == 0) rowsum[F.rsoff + (int64_t)itm.slab * L + p] = rowacc;
  }

  // column partials: fold the row slots of the wave, then the four waves
#pragma unroll
  for (int v = 0; v < MAXVPL; ++v)
#pragma unroll
    for (int e = 0; e < W; ++e) {
      double t = colacc[v][e];
      for (int off = LR; off < 64; off <<= 1) t += __shfl_xor(t, off, 64);
      colacc[v][e] = t;
    }
  if (slot == 0) {
#pragma unroll
    for (int v = 0; v < MAXVPL; ++v)
#pragma unroll
      for (int e = 0; e < W; ++e) {
        const int q = ((lin + (v << lrs)) * W) + e;
        if (v < vpl && q < L) lds_col[wave * (64 * MAXVPL * W) + q] = colacc[v][e];
      }
  }
  __syncthreads();
  double* cpo = colpart + F.cpoff + ((int64_t)itm.slab * F.nchunk + itm.chunk) * L;
  for (int q = threadIdx.x; q < L; q += kWG) {
    const int S = 64 * MAXVPL * W;
    cpo[q] = (lds_col[q] + lds_col[S + q]) + (lds_col[2 * S + q] + lds_col[3 * S + q]);
  }
  if (mode == MODE_CHECK) {
    double* ko = kitem + (int64_t)blockIdx.x * kKI;
    const double r_d = block_sum(kd, red);
    const double r_c = block_sum(kc, red);
    const double r_x = block_sum(kx, red);
    const double r_z = block_sum(kz, red);
    const double r_cx = block_sum(kcx, red);
    const double r_fp = block_sum(kfp, red);
    if (threadIdx.x == 0) {
      ko[KI_DUAL] = r_d;
      ko[KI_COMP] = r_c;
      ko[KI_XX] = r_x;
      ko[KI_ZZ] = r_z;
      ko[KI_CX] = r_cx;
      ko[KI_FP] = r_fp;
    }
  }
}

// ---------------------------------------------------------------------------
// Pair reduce: R = b/sigma - A(s - c) from the slab sums, plus the block sums
// of the structured solve (S1part, a_j, b1_j, PR3) and, on check passes, the
// KKT partials.  Block b of a pair owns F1 slabs j in [b*jpb, ...) and F2 slabs
// k in [b*kpb, ...).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_pair_reduce(
    const PBlock* __restrict__ blocks, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, const double* __restrict__ rowsum,
    const double* __restrict__ colpart, const double* __restrict__ rowsum_prev,
    const double* __restrict__ colpart_prev, const double* __restrict__ kitem,
    const double* __restrict__ ab, double* __restrict__ arr, double* __restrict__ vec) {
  __shared__ double S1loc[kMaxSide];
  __shared__ double red[4];
  const PBlock pbk = blocks[blockIdx.x];
  const PairCtl* cp = ctl + pbk.pair;
  if (cp->status != ST_RUNNING) return;
  const int mode = cp->mode;
  if (mode == MODE_IDLE) return;
  const PairGeo G = geo[pbk.pair];
  const int m = G.m, n = G.n, b = pbk.blk, t = threadIdx.x;
  const double isg = 1.0 / cp->sigma;
  const FamGeo F1 = G.f[0], F2 = G.f[1];
  const double* mu1T = arr + arr_mu1T(G);
  const double* mu2 = arr + arr_mu2(G);
  double* R1 = arr + arr_R1(G);
  double* R2 = arr + arr_R2(G);
  double* R3T = arr + arr_R3T(G);
  const int j0 = b * G.jpb, j1 = min(n, j0 + G.jpb);
  const int k0 = b * G.kpb, k1 = min(m, k0 + G.kpb);

  for (int k = t; k < m; k += kWG) S1loc[k] = 0.0;
  for (int j = j0; j < j1; ++j) {
    double sr1 = 0.0, sr2 = 0.0;
    for (int k = t; k < m; k += kWG) {
      const double rs1 = rowsum[F1.rsoff + (int64_t)j * m + k];
      const double rs2 = rowsum[F2.rsoff + (int64_t)k * n + j];
      const double r1 = -((rs1 - cost_rowsum(m, k)) - (rs2 - cost_rowsum(n, j)));
      R1[(int64_t)j * m + k] = r1;
      S1loc[k] += r1;
      sr1 += r1;
    }
    for (int i = t; i < m; i += kWG) {
      double cs = 0.0;
      const double* cpj = colpart + F1.cpoff + (int64_t)j * F1.nchunk * m + i;
      for (int c = 0; c < F1.nchunk; ++c) cs += cpj[(int64_t)c * m];
      const double r2 = mu1T[(int64_t)j * m + i] * isg - (cs - cost_rowsum(m, i));
      R2[(int64_t)j * m + i] = r2;
      sr2 += r2;
    }
    const double s1 = block_sum(sr1, red);
    const double s2 = block_sum(sr2, red);
    if (t == 0) {
      vec[vec_b1(G) + j] = s1;
      vec[vec_a(G) + j] = s2;
    }
  }
  __syncthreads();
  for (int k = t; k < m; k += kWG) vec[vec_S1(G) + (int64_t)b * m + k] = S1loc[k];
  for (int k = k0; k < k1; ++k) {
    double sr3 = 0.0;
    for (int l = t; l < n; l += kWG) {
      double r3 = 0.0;
      if (!(k == m - 1 && l == n - 1)) {
        double cs = 0.0;
        const double* cpk = colpart + F2.cpoff + (int64_t)k * F2.nchunk * n + l;
        for (int c = 0; c < F2.nchunk; ++c) cs += cpk[(int64_t)c * n];
        r3 = mu2[(int64_t)k * n + l] * isg - (cs - cost_rowsum(n, l));
      }
      R3T[(int64_t)k * n + l] = r3;
      sr3 += r3;
    }
    const double s3 = block_sum(sr3, red);
    if (t == 0) vec[vec_PR3(G) + k] = s3;
  }

  if (mode != MODE_CHECK) return;
  // ---- check pass: KKT partials of w_bar^k -------------------------------
  double part[kKI] = {0, 0, 0, 0, 0, 0, 0, 0};
  {
    const int i0 = G.item0 + b * G.ipb;
    const int i1 = min(G.item0 + G.nitem, i0 + G.ipb);
    for (int it = i0 + t; it < i1; it += kWG)
      for (int q = 0; q < 6; ++q) part[q] += kitem[(int64_t)it * kKI + q];
  }
  // primal residual A xbar - b with xbar = sigma (s - g): the sums of s^k are
  // the previous pass's sums; the sums of g over a slab row / column follow
  // from alpha, beta and their per-slab totals (written by the solve).
  const double sg = cp->sigma;
  double prim = 0.0, by = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double* al = ab + F1.aboff + (int64_t)j * 2 * m;
    const double* be = al + m;
    const double sa = ab[F1.sumoff + 2 * (int64_t)j], sb = ab[F1.sumoff + 2 * (int64_t)j + 1];
    for (int k = t; k < m; k += kWG) {
      // row k of F1^(j) and row j of F2^(k) share the conservation row (j,k)
      const double* al2 = ab + F2.aboff + (int64_t)k * 2 * n;
      const double sb2 = ab[F2.sumoff + 2 * (int64_t)k + 1];
      const double x1 = sg * (rowsum_prev[F1.rsoff + (int64_t)j * m + k] -
                              (cost_rowsum(m, k) - m * al[k] - sb));
      const double x2 = sg * (rowsum_prev[F2.rsoff + (int64_t)k * n + j] -
                              (cost_rowsum(n, j) - n * al2[j] - sb2));
      const double r = x1 - x2;
      prim += r * r;
    }
    for (int i = t; i < m; i += kWG) {
      double cs = 0.0;
      const double* cpj = colpart_prev + F1.cpoff + (int64_t)j * F1.nchunk * m + i;
      for (int c = 0; c < F1.nchunk; ++c) cs += cpj[(int64_t)c * m];
      const double x = sg * (cs - (cost_rowsum(m, i) - sa - m * be[i]));
      const double r = x - mu1T[(int64_t)j * m + i];
      prim += r * r;
      by += mu1T[(int64_t)j * m + i] * be[i];
    }
  }
  for (int k = k0; k < k1; ++k) {
    const double* al = ab + F2.aboff + (int64_t)k * 2 * n;
    const double* be = al + n;
    const double sa = ab[F2.sumoff + 2 * (int64_t)k];
    for (int l = t; l < n; l += kWG) {
      if (k == m - 1 && l == n - 1) continue;
      double cs = 0.0;
      const double* cpk = colpart_prev + F2.cpoff + (int64_t)k * F2.nchunk * n + l;
      for (int c = 0; c < F2.nchunk; ++c) cs += cpk[(int64_t)c * n];
      const double x = sg * (cs - (cost_rowsum(n, l) - sa - n * be[l]));
      const double r = x - mu2[(int64_t)k * n + l];
      prim += r * r;
      by += mu2[(int64_t)k * n + l] * be[l];
    }
  }
  double* kp = vec + vec_kpart(G) + (int64_t)b * kKP;
  double outv[kKP];
  for (int q = 0; q < 6; ++q) outv[q] = block_sum(part[q], red);
  outv[KP_PRIM] = block_sum(prim, red);
  outv[KP_BY] = block_sum(by, red);
  if (t == 0)
    for (int q = 0; q < 8; ++q) kp[q] = outv[q];
}

// Row-k alpha/beta of slab F2^(k) are -y1[.][k] and y3[.][k]; y1 entries are
// recomputed from the same formula as the F1 side (identical inputs).
__device__ inline double y1_entry(const double* R1, const double* a, const double* PR3,
                                  const double* tq, const double* rsj, int m, int n,
                                  int j, int k) {
  const double dm = (double)m, dn = (double)n;
  const double rh = R1[(int64_t)j * m + k] - a[j] / dm + PR3[k] / dn;
  return (rh + tq[k] + rsj[j] / dn) / (dm + dn);
}

// ---------------------------------------------------------------------------
// Pair solve.  Every block of a pair first reproduces the same decision from
// the check partials (fixed summation order), then, unless the pair stops or
// restarts, solves A A^T ybar = R in the Schur-complement form:
//   Rhat1^j = R1^j - (1^T R2^j / m) 1 + PR3 / n,  S = sum_j Rhat1^j,
//   (D - 1 1^T) t = S with D = diag(m, .., m, m+1)   (t = sum_j y1^j),
//   y1^j = (I + 1 1^T / n)(Rhat1^j + Q t)/(m+n),  Q = I - e_m e_m^T / n,
//   y2^j = (R2^j - (1^T y1^j) 1)/m,  y3^l = (R3^l + t)/n.
// Block 0 writes the control block of the next pass (other parity).
// ---------------------------------------------------------------------------
__device__ void decide(const PairGeo& G, const PairCtl& c, const double* vec, PairCtl& nx,
                       bool& solve) {
  nx = c;
  solve = false;
  const bool fixed = (c.flags & 2) != 0;
  const bool restart_on = (c.flags & 1) != 0 && !fixed;
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
      double acc[kKP];
      for (int q = 0; q < kKP; ++q) acc[q] = 0.0;
      const double* kp = vec + vec_kpart(G);
      for (int b = 0; b < G.nblk; ++b)
        for (int q = 0; q < 8; ++q) acc[q] += kp[(int64_t)b * kKP + q];
      const double nx2 = sqrt(acc[KP_XX]), nz2 = sqrt(acc[KP_ZZ]);
      nx.res_d = sqrt(acc[KP_DUAL]) / (1.0 + G.norm_c);
      nx.res_c = sqrt(acc[KP_COMP]) / (1.0 + nx2 + nz2);
      nx.res_p = sqrt(acc[KP_PRIM]) / (1.0 + G.norm_b);
      nx.kkt = fmax(nx.res_d, fmax(nx.res_c, nx.res_p));
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
      } else if (c.tol > 0 && nx.kkt <= c.tol) {
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
          // src keeps s^k for the restart pass
          return;
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
  nx.lam = 1.0 / (double)(nx.k + 2);
  // fixed mode: plain updates, then one check pass at it == K that only
  // evaluates w_bar^K
  nx.mode = fixed ? (nx.it >= c.max_iter ? MODE_CHECK : MODE_NORMAL)
                  : ((nx.k % c.T == 0 || nx.it >= c.max_iter) ? MODE_CHECK : MODE_NORMAL);
  nx.dst = (nx.mode == MODE_CHECK || nx.src == 2) ? (nx.src == 0 ? 1 : 0) : nx.src;
}

__device__ void solve_blocks(const PairGeo& G, int b, const double* arr, double* vec,
                             double* ab, double* tq_lds, double* red) {
  const int m = G.m, n = G.n, t = threadIdx.x;
  const double dm = (double)m, dn = (double)n;
  const double* R1 = arr + arr_R1(G);
  const double* R2 = arr + arr_R2(G);
  const double* R3T = arr + arr_R3T(G);
  const double* a = vec + vec_a(G);
  const double* b1 = vec + vec_b1(G);
  const double* PR3 = vec + vec_PR3(G);
  const double* S1 = vec + vec_S1(G);
  // totals over j of a_j, and over k of PR3
  double sa = 0.0;
  for (int j = t; j < n; j += kWG) sa += a[j];
  sa = block_sum(sa, red);
  double sp = 0.0;
  for (int k = t; k < m; k += kWG) sp += PR3[k];
  sp = block_sum(sp, red);
  // S and D^{-1} S
  double u = 0.0;
  for (int k = t; k < m; k += kWG) {
    double s = 0.0;
    for (int bb = 0; bb < G.nblk; ++bb) s += S1[(int64_t)bb * m + k];
    s = s - sa / dm + PR3[k];
    const double dk = (k == m - 1) ? dm + 1.0 : dm;
    tq_lds[k] = s / dk;
    u += s / dk;
  }
  u = block_sum(u, red);
  // t = D^{-1} S + m(m+1) (1^T D^{-1} S) D^{-1} 1 ;  Qt = t - e_m t_m / n
  double sq = 0.0;
  for (int k = t; k < m; k += kWG) {
    const double dk = (k == m - 1) ? dm + 1.0 : dm;
    const double tk = tq_lds[k] + dm * (dm + 1.0) * u / dk;
    tq_lds[kMaxSide + k] = tk;                       // t
    const double q = (k == m - 1) ? tk - tk / dn : tk;  // Q t
    tq_lds[k] = q;
    sq += q;
  }
  sq = block_sum(sq, red);
  __syncthreads();
  const double* tq = tq_lds;                 // Q t
  const double* tt = tq_lds + kMaxSide;      // t
  // rsj[j] = 1^T (Rhat1^j + Q t) = b1_j - a_j + sum(PR3)/n + sum(Qt)
  double* rsj = tq_lds + 2 * kMaxSide;
  for (int j = t; j < n; j += kWG) rsj[j] = b1[j] - a[j] + sp / dn + sq;
  __syncthreads();
  const FamGeo F1 = G.f[0], F2 = G.f[1];
  const int j0 = b * G.jpb, j1 = min(n, j0 + G.jpb);
  const int k0 = b * G.kpb, k1 = min(m, k0 + G.kpb);
  for (int j = j0; j < j1; ++j) {
    double* al = ab + F1.aboff + (int64_t)j * 2 * m;
    double* be = al + m;
    double sa = 0.0, sb = 0.0;
    for (int k = t; k < m; k += kWG) {
      const double v = y1_entry(R1, a, PR3, tq, rsj, m, n, j, k);
      al[k] = v;
      sa += v;
    }
    // 1^T y1^j = rsj / n
    for (int i = t; i < m; i += kWG) {
      const double v = (R2[(int64_t)j * m + i] - rsj[j] / dn) / dm;
      be[i] = v;
      sb += v;
    }
    sa = block_sum(sa, red);
    sb = block_sum(sb, red);
    if (t == 0) {
      ab[F1.sumoff + 2 * (int64_t)j] = sa;
      ab[F1.sumoff + 2 * (int64_t)j + 1] = sb;
    }
  }
  for (int k = k0; k < k1; ++k) {
    double* al = ab + F2.aboff + (int64_t)k * 2 * n;
    double* be = al + n;
    double sa = 0.0, sb = 0.0;
    for (int j = t; j < n; j += kWG) {
      const double v = -y1_entry(R1, a, PR3, tq, rsj, m, n, j, k);
      al[j] = v;
      sa += v;
    }
    for (int l = t; l < n; l += kWG) {
      const double v =
          (k == m - 1 && l == n - 1) ? 0.0 : (R3T[(int64_t)k * n + l] + tt[k]) / dn;
      be[l] = v;
      sb += v;
    }
    sa = block_sum(sa, red);
    sb = block_sum(sb, red);
    if (t == 0) {
      ab[F2.sumoff + 2 * (int64_t)k] = sa;
      ab[F2.sumoff + 2 * (int64_t)k + 1] = sb;
    }
  }
}

__global__ __launch_bounds__(kWG) void k_pair_solve(const PBlock* __restrict__ blocks,
                                                    const PairGeo* __restrict__ geo,
                                                    const PairCtl* __restrict__ ctl,
                                                    PairCtl* __restrict__ ctl_next,
                                                    const double* __restrict__ arr,
                                                    double* __restrict__ vec,
                                                    double* __restrict__ ab) {
  __shared__ double tq_lds[3 * kMaxSide];
  __shared__ double red[4];
  const PBlock pbk = blocks[blockIdx.x];
  const PairCtl c = ctl[pbk.pair];
  if (c.status != ST_RUNNING || c.mode == MODE_IDLE) {
    if (pbk.blk == 0 && threadIdx.x == 0) ctl_next[pbk.pair] = c;
    return;
  }
  const PairGeo G = geo[pbk.pair];
  PairCtl nx;
  bool solve;
  decide(G, c, vec, nx, solve);
  if (solve) solve_blocks(G, pbk.blk, arr, vec, ab, tq_lds, red);
  if (pbk.blk == 0 && threadIdx.x == 0) ctl_next[pbk.pair] = nx;
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
                         double* __restrict__ sout) {
  const PairGeo G = geo[pair];
  const PairCtl c = ctl[pair];
  const int m = G.m, n = G.n;
  const int64_t N1 = (int64_t)m * m * n, N = N1 + (int64_t)m * n * n;
  const T* s = pick<const T>(sb0, sb1, sb2, c.src);
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
    const double sv = (double)s[F.soff + ((int64_t)slab * L + p) * F.P + q];
    const double* al = ab + F.aboff + (int64_t)slab * 2 * L;
    const double d = (double)(p - q);
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

// Block sums of the solve from stored R arrays (hot_aat_solve path).
__global__ __launch_bounds__(kWG) void k_pair_sums_from_R(const PBlock* __restrict__ blocks,
                                                          const PairGeo* __restrict__ geo,
                                                          const double* __restrict__ arr,
                                                          double* __restrict__ vec) {
  __shared__ double S1loc[kMaxSide];
  __shared__ double red[4];
  const PBlock pbk = blocks[blockIdx.x];
  const PairGeo G = geo[pbk.pair];
  const int m = G.m, n = G.n, b = pbk.blk, t = threadIdx.x;
  const double* R1 = arr + arr_R1(G);
  const double* R2 = arr + arr_R2(G);
  const double* R3T = arr + arr_R3T(G);
  const int j0 = b * G.jpb, j1 = min(n, j0 + G.jpb);
  const int k0 = b * G.kpb, k1 = min(m, k0 + G.kpb);
  for (int k = t; k < m; k += kWG) S1loc[k] = 0.0;
  for (int j = j0; j < j1; ++j) {
    double sr1 = 0.0, sr2 = 0.0;
    for (int k = t; k < m; k += kWG) {
      const double r1 = R1[(int64_t)j * m + k];
      S1loc[k] += r1;
      sr1 += r1;
    }
    for (int i = t; i < m; i += kWG) sr2 += R2[(int64_t)j * m + i];
    const double s1 = block_sum(sr1, red);
    const double s2 = block_sum(sr2, red);
    if (t == 0) {
      vec[vec_b1(G) + j] = s1;
      vec[vec_a(G) + j] = s2;
    }
  }
  __syncthreads();
  for (int k = t; k < m; k += kWG) vec[vec_S1(G) + (int64_t)b * m + k] = S1loc[k];
  for (int k = k0; k < k1; ++k) {
    double sr3 = 0.0;
    for (int l = t; l < n; l += kWG) sr3 += R3T[(int64_t)k * n + l];
    const double s3 = block_sum(sr3, red);
    if (t == 0) vec[vec_PR3(G) + k] = s3;
  }
}

__global__ __launch_bounds__(kWG) void k_pair_solve_only(const PBlock* __restrict__ blocks,
                                                         const PairGeo* __restrict__ geo,
                                                         const double* __restrict__ arr,
                                                         double* __restrict__ vec,
                                                         double* __restrict__ ab) {
  __shared__ double tq_lds[3 * kMaxSide];
  __shared__ double red[4];
  const PBlock pbk = blocks[blockIdx.x];
  const PairGeo G = geo[pbk.pair];
  solve_blocks(G, pbk.blk, arr, vec, ab, tq_lds, red);
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage inside the library).
// ---------------------------------------------------------------------------


template <typename T, int V>
static void launch_slab(const LaunchArgs& a, int par, hipStream_t st) {
  hipLaunchKernelGGL((k_slab_pass<T, V>), dim3(a.nitems), dim3(kWG), 0, st, a.items, a.geo,
                     a.ctl[par], (T*)a.sb[0], (T*)a.sb[1], (T*)a.sb[2], a.ab, a.rowsum[par],
                     a.colpart[par], a.kitem);
}

template <typename T>
static void launch_slab_t(const LaunchArgs& a, int par, hipStream_t st) {
  if (a.maxvpl <= 1) launch_slab<T, 1>(a, par, st);
  else if (a.maxvpl <= 2) launch_slab<T, 2>(a, par, st);
  else if (a.maxvpl <= 4) launch_slab<T, 4>(a, par, st);
  else launch_slab<T, 8>(a, par, st);
}

// One iteration: slab pass, pair reduce, pair solve.  Reads ctl[par], writes ctl[1-par].
void launch_iteration(const LaunchArgs& a, int par, hipStream_t st) {
  if (a.fp32) launch_slab_t<float>(a, par, st);
  else launch_slab_t<double>(a, par, st);
  hipLaunchKernelGGL(k_pair_reduce, dim3(a.nblocks), dim3(kWG), 0, st, a.blocks, a.geo,
                     a.ctl[par], a.rowsum[par], a.colpart[par], a.rowsum[1 - par],
                     a.colpart[1 - par], a.kitem, a.ab, a.arr, a.vec);
  hipLaunchKernelGGL(k_pair_solve, dim3(a.nblocks), dim3(kWG), 0, st, a.blocks, a.geo,
                     a.ctl[par], a.ctl[1 - par], a.arr, a.vec, a.ab);
}

void launch_hist_stats_multi(const double* const* ptrs, const int64_t* lens, int count,
                             double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_hist_stats_multi, dim3(count), dim3(kWG), 0, st, ptrs, lens, out);
}

void launch_setup_mu(const double* mu1, const double* mu2, int m, int n, double* mu1T,
                     double* mu2c, hipStream_t st) {
  const int64_t M = (int64_t)m * n;
  const int grid = (int)std::min<int64_t>((M + kWG - 1) / kWG, 4096);
  hipLaunchKernelGGL(k_setup_mu, dim3(grid), dim3(kWG), 0, st, mu1, mu2, m, n, mu1T, mu2c);
}

void launch_export(const LaunchArgs& a, int par, int pair, int64_t N, double* xbar,
                   double* zbar, double* sout, hipStream_t st) {
  const int grid = (int)std::min<int64_t>((N + kWG - 1) / kWG, 65536);
  if (a.fp32)
    hipLaunchKernelGGL(k_export<float>, dim3(grid), dim3(kWG), 0, st, a.geo, a.ctl[par], pair,
                       (const float*)a.sb[0], (const float*)a.sb[1], (const float*)a.sb[2], a.ab,
                       xbar, zbar, sout);
  else
    hipLaunchKernelGGL(k_export<double>, dim3(grid), dim3(kWG), 0, st, a.geo, a.ctl[par], pair,
                       (const double*)a.sb[0], (const double*)a.sb[1], (const double*)a.sb[2],
                       a.ab, xbar, zbar, sout);
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
  hipLaunchKernelGGL(k_pair_solve_only, dim3(a.nblocks), dim3(kWG), 0, st, a.blocks, a.geo,
                     a.arr, a.vec, a.ab);
}

}  // namespace hot

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
  typedef float native __attribute__((ext_vector_type(4)));
};
template <>
struct VecT<double> {
  static constexpr int W = 2;
  typedef double2 type;
  typedef double native __attribute__((ext_vector_type(2)));
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
// a wave covers 64/LR rows per step, the four waves interleave, and two
// steps are loaded before either is computed.  Column sums stay in FP64
// registers for the whole chunk; row sums are finished with DPP moves inside
// the wave (the sum lands in the last lane of each LR-lane group).
// The pass is specialised at compile time on its mode and on where the
// Halpern anchor comes from, so the element loop has no branches.
// ---------------------------------------------------------------------------
template <int CTRL, int RM = 0xf>
__device__ inline double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  int lo = (int)b, hi = (int)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, RM, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, RM, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over aligned groups of LR lanes (LR a power of two <= 64); valid in
// the last lane of each group.
__device__ inline double group_sum(double v, int LR) {
  if (LR >= 2) v += dpp_mov<0xB1>(v);        // quad_perm [1,0,3,2]
  if (LR >= 4) v += dpp_mov<0x4E>(v);        // quad_perm [2,3,0,1]
  if (LR >= 8) v += dpp_mov<0x141>(v);       // row_half_mirror
  if (LR >= 16) v += dpp_mov<0x140>(v);      // row_mirror
  if (LR >= 32) v += dpp_mov<0x142, 0xA>(v); // row_bcast:15 into rows 1, 3
  if (LR >= 64) v += dpp_mov<0x143, 0xC>(v); // row_bcast:31 into rows 2, 3
  return v;
}

enum { ANC_ZERO = 0, ANC_SAME = 1, ANC_SEP = 2 };

struct SlabCtx {
  int L, P, r0, r1, lrs, vpl, lin, slot, wave, lane;
  double lam, oml, sigma;
};

template <typename T, int MAXVPL, int MODE, int ANC, int U, int C>
__device__ inline void slab_rows(const SlabCtx& x, const T* __restrict__ src,
                                 T* __restrict__ dst, const T* __restrict__ anc,
                                 const double* __restrict__ alpha, const double* __restrict__ bl,
                                 const double* __restrict__ lx,
                                 double (&colacc)[MAXVPL][VecT<T>::W], double* __restrict__ rowsum,
                                 double (&kk)[6]) {
  constexpr int W = VecT<T>::W;
  typedef typename VecT<T>::type VT;
  const int LR = 1 << x.lrs, rpw = 64 >> x.lrs;
  const int L = x.L, P = x.P;
  constexpr int UR = U & 3;
  for (int pb = x.r0 + x.wave * rpw; pb < x.r1; pb += 4 * UR * rpw) {
    int prow[UR];
    bool rvv[UR];
    VT xs[UR][MAXVPL], xa[UR][MAXVPL];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      prow[u] = pb + u * 4 * rpw + x.slot;
      rvv[u] = prow[u] < x.r1;
#pragma unroll
      for (int v = 0; v < MAXVPL; ++v) {
        const int q0 = (x.lin + (v << x.lrs)) * W;
        if (v < x.vpl && rvv[u] && q0 < L) {
          xs[u][v] = *reinterpret_cast<const VT*>(src + (int64_t)prow[u] * P + q0);
          if (ANC == ANC_SEP) xa[u][v] = *reinterpret_cast<const VT*>(anc + (int64_t)prow[u] * P + q0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int p = prow[u];
      const bool rv = rvv[u];
      const double ap = rv ? alpha[p] : 0.0;
      const double xp = (C && rv) ? lx[p] : 0.0;  // row position (non-uniform bins)
      double rowacc = 0.0;
#pragma unroll
      for (int v = 0; v < MAXVPL; ++v) {
        const int q0 = (x.lin + (v << x.lrs)) * W;
        if (v < x.vpl && rv && q0 < L) {
          VT out;
          const double d0 = (double)(p - q0);
#pragma unroll
          for (int e = 0; e < W; ++e) {
            const bool ok = (q0 + e) < L;
            const double s = (double)vget(xs[u][v], e);
            const double d = C ? xp - lx[q0 + e] : d0 - (double)e;
            const double g = d * d - (ap + bl[q0 + e]);
            double o;
            if (MODE == MODE_RESTART) {
              o = fmax(s - g, g);
            } else {
              const double sh = fabs(s - 2.0 * g);
              if (ANC == ANC_ZERO) o = x.oml * sh;
              else if (ANC == ANC_SAME) o = x.lam * s + x.oml * sh;
              else o = x.lam * (double)vget(xa[u][v], e) + x.oml * sh;
              if (MODE == MODE_CHECK) {
                const double xb = x.sigma * (s - g);
                const double zb = fmax(0.0, 2.0 * g - s);
                const double dr = zb - g;
                const double mn = fmin(xb, zb);
                const double fr = s - sh;
                kk[KI_DUAL] += ok ? dr * dr : 0.0;
                kk[KI_COMP] += ok ? mn * mn : 0.0;
                kk[KI_XX] += ok ? xb * xb : 0.0;
                kk[KI_ZZ] += ok ? zb * zb : 0.0;
                kk[KI_CX] += ok ? d * d * xb : 0.0;
                kk[KI_FP] += ok ? fr * fr : 0.0;
              }
            }
            const T st = ok ? (T)o : (T)0;
            const double sd = (double)st;
            rowacc += sd;
            colacc[v][e] += sd;
            vset(out, e, st);
          }
          if (U & 4)
            __builtin_nontemporal_store(
                __builtin_bit_cast(typename VecT<T>::native, out),
                reinterpret_cast<typename VecT<T>::native*>(dst + (int64_t)p * P + q0));
          else
            *reinterpret_cast<VT*>(dst + (int64_t)p * P + q0) = out;
        }
      }
      rowacc = group_sum(rowacc, LR);
      if (rv && x.lin == LR - 1) rowsum[p] = rowacc;
    }
  }
}

// HEAVY = 0: plain update passes; HEAVY = 1: check and restart passes.  Both
// kernels are launched every iteration; a workgroup whose pair is in the
// other kind of pass exits at once.
template <typename T, int MAXVPL, int HEAVY, int U, int C>
__device__ inline void slab_item(
    int item, const SlabItem* __restrict__ items, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, T* __restrict__ sb0, T* __restrict__ sb1,
    T* __restrict__ sb2, const double* __restrict__ ab, double* __restrict__ rowsum,
    double* __restrict__ colpart, double* __restrict__ kitem,
    unsigned long long* __restrict__ bytes_ctr, double* lds_col, double* lds_beta, double* lds_x,
    double* red) {
  constexpr int W = VecT<T>::W;
  constexpr int S = 64 * MAXVPL * W;
  const SlabItem itm = items[item];
  const PairCtl* cp = ctl + itm.pair;
  const int status = cp->status;
  const int mode = cp->mode;
  if (status != ST_RUNNING) return;
  if (HEAVY ? (mode != MODE_CHECK && mode != MODE_RESTART) : (mode != MODE_NORMAL)) return;
  // (uniform per workgroup: every thread reads the same control block)
  const FamGeo F = geo[itm.pair].f[itm.fam];
  SlabCtx x;
  x.L = F.L;
  x.P = F.P;
  x.r0 = itm.chunk * F.rpc;
  x.r1 = min(F.L, x.r0 + F.rpc);
  x.lrs = F.lrs;
  x.vpl = F.vpl;
  x.lane = threadIdx.x & 63;
  x.wave = threadIdx.x >> 6;
  x.slot = x.lane >> x.lrs;
  x.lin = x.lane & ((1 << x.lrs) - 1);
  x.lam = cp->lam;
  x.oml = 1.0 - cp->lam;
  x.sigma = cp->sigma;
  const int L = F.L;
  const int64_t soff = F.soff + (int64_t)itm.slab * L * F.P;
  const int src_i = cp->src, anc_i = cp->anc;
  const int dst_i = (mode == MODE_RESTART) ? 2 : cp->dst;
  const T* src = pick<T>(sb0, sb1, sb2, src_i) + soff;
  T* dst = pick<T>(sb0, sb1, sb2, dst_i) + soff;
  const int anc_kind =
      (mode == MODE_RESTART || anc_i < 0) ? ANC_ZERO : (anc_i == src_i ? ANC_SAME : ANC_SEP);
  const T* anc = anc_kind == ANC_SEP ? pick<T>(sb0, sb1, sb2, anc_i) + soff : src;
  const double* alpha = ab + F.aboff + (int64_t)itm.slab * 2 * L;
  const double* beta = alpha + L;
  double* rs = rowsum + F.rsoff + (int64_t)itm.slab * L;
  // beta in LDS (zero in the padding columns); the barrier also keeps the
  // previous item's readers of lds_col / lds_beta behind us
  __syncthreads();
  for (int q = threadIdx.x; q < F.P; q += kWG) lds_beta[q] = q < L ? beta[q] : 0.0;
  if (C) {
    const double* X = fam_x(ab, F);
    for (int q = threadIdx.x; q < F.P; q += kWG) lds_x[q] = q < L ? X[q] : 0.0;
  }
  __syncthreads();

  double colacc[MAXVPL][W];
#pragma unroll
  for (int v = 0; v < MAXVPL; ++v)
#pragma unroll
    for (int e = 0; e < W; ++e) colacc[v][e] = 0.0;
  double kk[6] = {0, 0, 0, 0, 0, 0};
  if (!HEAVY) {
    if (anc_kind == ANC_ZERO)
      slab_rows<T, MAXVPL, MODE_NORMAL, ANC_ZERO, U, C>(x, src, dst, anc, alpha, lds_beta, lds_x, colacc, rs, kk);
    else if (anc_kind == ANC_SAME)
      slab_rows<T, MAXVPL, MODE_NORMAL, ANC_SAME, U, C>(x, src, dst, anc, alpha, lds_beta, lds_x, colacc, rs, kk);
    else
      slab_rows<T, MAXVPL, MODE_NORMAL, ANC_SEP, U, C>(x, src, dst, anc, alpha, lds_beta, lds_x, colacc, rs, kk);
  } else if (mode == MODE_CHECK) {
    if (anc_kind == ANC_ZERO)
      slab_rows<T, MAXVPL, MODE_CHECK, ANC_ZERO, U, C>(x, src, dst, anc, alpha, lds_beta, lds_x, colacc, rs, kk);
    else if (anc_kind == ANC_SAME)
      slab_rows<T, MAXVPL, MODE_CHECK, ANC_SAME, U, C>(x, src, dst, anc, alpha, lds_beta, lds_x, colacc, rs, kk);
    else
      slab_rows<T, MAXVPL, MODE_CHECK, ANC_SEP, U, C>(x, src, dst, anc, alpha, lds_beta, lds_x, colacc, rs, kk);
  } else {
    slab_rows<T, MAXVPL, MODE_RESTART, ANC_ZERO, U, C>(x, src, dst, anc, alpha, lds_beta, lds_x, colacc, rs, kk);
  }

  // column partials: fold the row slots of the wave, then the four waves
  const int LR = 1 << x.lrs;
#pragma unroll
  for (int v = 0; v < MAXVPL; ++v)
#pragma unroll
    for (int e = 0; e < W; ++e) {
      double t = colacc[v][e];
      for (int off = LR; off < 64; off <<= 1) t += __shfl_xor(t, off, 64);
      colacc[v][e] = t;
    }
  if (x.slot == 0) {
#pragma unroll
    for (int v = 0; v < MAXVPL; ++v)
#pragma unroll
      for (int e = 0; e < W; ++e) {
        const int q = ((x.lin + (v << x.lrs)) * W) + e;
        if (v < x.vpl && q < L) lds_col[x.wave * S + q] = colacc[v][e];
      }
  }
  __syncthreads();
  double* cpo = colpart + F.cpoff + ((int64_t)itm.slab * F.nchunk + itm.chunk) * L;
  for (int q = threadIdx.x; q < L; q += kWG)
    cpo[q] = (lds_col[q] + lds_col[S + q]) + (lds_col[2 * S + q] + lds_col[3 * S + q]);
  if (threadIdx.x == 0 && bytes_ctr) {
    // algorithmic stream traffic of this item: read s (and the anchor when it
    // is a separate buffer), write the new state
    const int streams = anc_kind == ANC_SEP ? 3 : 2;
    atomicAdd(bytes_ctr, (unsigned long long)(x.r1 - x.r0) * L * sizeof(T) * streams);
  }
  if (HEAVY && mode == MODE_CHECK) {
    double* ko = kitem + (int64_t)item * kKI;
    double r[6];
    for (int q = 0; q < 6; ++q) r[q] = block_sum(kk[q], red);
    if (threadIdx.x == 0)
      for (int q = 0; q < 6; ++q) ko[q] = r[q];
  }
}

// One workgroup per item.
template <typename T, int MAXVPL, int HEAVY, int U, int C>
__global__ __launch_bounds__(kWG) void k_slab_pass(
    const SlabItem* __restrict__ items, int nitems, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, T* __restrict__ sb0, T* __restrict__ sb1,
    T* __restrict__ sb2, const double* __restrict__ ab, double* __restrict__ rowsum,
    double* __restrict__ colpart, double* __restrict__ kitem,
    unsigned long long* __restrict__ bytes_ctr) {
  constexpr int W = VecT<T>::W;
  constexpr int S = 64 * MAXVPL * W;
  __shared__ double lds_col[4 * S];
  __shared__ double lds_beta[S];
  __shared__ double lds_x[C ? S : 1];
  __shared__ double red[4];
  if ((int)blockIdx.x < nitems)
    slab_item<T, MAXVPL, HEAVY, U, C>(blockIdx.x, items, geo, ctl, sb0, sb1, sb2, ab, rowsum,
                                      colpart, kitem, bytes_ctr, lds_col, lds_beta, lds_x, red);
}

// ---------------------------------------------------------------------------
// Pair reduce: R = b/sigma - A(s - c) from the slab sums, the totals the
// structured solve needs, and (check passes) the KKT partials.
//   kind 0, row block b: one wave per row j = 4b + w of R2 (and the total of
//           row j of the F1 row sums) and per row k = 4b + w of R3^T (and the
//           total of row k of the F2 row sums);
//   kind 1, strip s: u1[k] = sum_j rs1[j][k] for 64 columns k (lane per column);
//   kind 2, strip s: u2[j] = sum_k rs2[k][j] for 64 columns j.
// Every access is along a row.  R1 itself is never stored: the solve reads
// it straight from the two row-sum arrays, tile by tile.
// With C_L(p) = sum_q (X_p - X_q)^2 and CC_L = sum_p C_L(p) from the family's
// cost table (X_p = p on the uniform grid):
//   R1[j][k] = -(rs1[j][k] - C_m(k)) + (rs2[k][j] - C_n(j)),
//   1^T R1^j = -(tot1[j] - CC_m) + (u2[j] - m C_n(j)),
//   sum_j R1[j][k] = -(u1[k] - n C_m(k)) + (tot2[k] - CC_n).
// ---------------------------------------------------------------------------
__device__ inline double dinv(int m, int k) { return (k == m - 1) ? 1.0 / (m + 1.0) : 1.0 / m; }

__global__ __launch_bounds__(kWG) void k_pair_reduce(
    const PBlock* __restrict__ blocks, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, const double* __restrict__ rowsum,
    const double* __restrict__ colpart, const double* __restrict__ rowsum_prev,
    const double* __restrict__ colpart_prev, const double* __restrict__ kitem,
    const double* __restrict__ ab, double* __restrict__ arr, double* __restrict__ vec) {
  __shared__ double wred[4][kKP];
  __shared__ double strip[4][64];
  const PBlock pbk = blocks[blockIdx.x];
  const PairCtl* cp = ctl + pbk.pair;
  if (cp->status != ST_RUNNING) return;
  const int mode = cp->mode;
  if (mode == MODE_IDLE) return;
  const PairGeo G = geo[pbk.pair];
  const int m = G.m, n = G.n, b = pbk.blk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const FamGeo F1 = G.f[0], F2 = G.f[1];
  if (pbk.kind != 0) {
    // column totals of a row-sum array: lane = column, waves split the rows
    const bool s1 = pbk.kind == 1;
    const int ncol = s1 ? m : n, nrow = s1 ? n : m;
    const double* rs = s1 ? rowsum + F1.rsoff : rowsum + F2.rsoff;  // [nrow][ncol]
    const int col = 64 * b + lane;
    double acc = 0.0;
    if (col < ncol)
      for (int r = wave; r < nrow; r += 4) acc += rs[(int64_t)r * ncol + col];
    strip[wave][lane] = acc;
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
  const double isg = 1.0 / cp->sigma;
  const double* mu1T = arr + arr_mu1T(G);
  const double* mu2 = arr + arr_mu2(G);
  double* R2 = arr + arr_R2(G);
  double* R3T = arr + arr_R3T(G);
  const int j = 4 * b + wave, k = 4 * b + wave;
  double p_sa = 0.0, p_sp = 0.0, p_u = 0.0;
  if (j < n) {
    double sr2 = 0.0, t1 = 0.0;
    const double* cpj = colpart + F1.cpoff + (int64_t)j * F1.nchunk * m;
    for (int i = lane; i < m; i += 64) {
      double cs = 0.0;
      for (int c = 0; c < F1.nchunk; ++c) cs += cpj[(int64_t)c * m + i];
      const double r2 = mu1T[(int64_t)j * m + i] * isg - (cs - fam_cr(ab, F1, i));
      R2[(int64_t)j * m + i] = r2;
      sr2 += r2;
      t1 += rowsum[F1.rsoff + (int64_t)j * m + i];  // row j of the F1 row sums
    }
    sr2 = wave_sum(sr2);
    t1 = wave_sum(t1);
    if (lane == 0) {
      vec[vec_a(G) + j] = sr2;
      vec[vec_tot1(G) + j] = t1;
    }
    p_sa = sr2;
  }
  if (k < m) {
    double s3 = 0.0, t2 = 0.0;
    const double* cpk = colpart + F2.cpoff + (int64_t)k * F2.nchunk * n;
    for (int l = lane; l < n; l += 64) {
      double r3 = 0.0;
      if (!(k == m - 1 && l == n - 1)) {
        double cs = 0.0;
        for (int c = 0; c < F2.nchunk; ++c) cs += cpk[(int64_t)c * n + l];
        r3 = mu2[(int64_t)k * n + l] * isg - (cs - fam_cr(ab, F2, l));
      }
      R3T[(int64_t)k * n + l] = r3;
      s3 += r3;
      t2 += rowsum[F2.rsoff + (int64_t)k * n + l];  // row k of the F2 row sums
    }
    s3 = wave_sum(s3);
    t2 = wave_sum(t2);
    if (lane == 0) {
      vec[vec_PR3(G) + k] = s3;
      vec[vec_tot2(G) + k] = t2;
    }
    p_sp = s3;
    p_u = ((t2 - fam_cc(ab, F2)) + s3) * dinv(m, k);
  }
  if (lane == 0) {
    wred[wave][0] = p_sa;
    wred[wave][1] = p_sp;
    wred[wave][2] = p_u;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int q = threadIdx.x;
    vec[vec_spart(G) + 4 * (int64_t)b + q] = (wred[0][q] + wred[1][q]) + (wred[2][q] + wred[3][q]);
  }
  if (mode != MODE_CHECK) return;

  // ---- check pass: KKT partials of w_bar^k -------------------------------
  double part[kKI] = {0, 0, 0, 0, 0, 0, 0, 0};
  {
    const int i0 = G.item0 + b * G.ipb;
    const int i1 = min(G.item0 + G.nitem, i0 + G.ipb);
    for (int it = i0 + (int)threadIdx.x; it < i1; it += kWG)
      for (int q = 0; q < 6; ++q) part[q] += kitem[(int64_t)it * kKI + q];
  }
  // primal residual A xbar - b, xbar = sigma (s - g): the sums of s^k are the
  // previous pass's sums; the sums of g over a slab row / column follow from
  // alpha, beta and their per-slab totals.
  const double sg = cp->sigma;
  double prim = 0.0, by = 0.0;
  if (j < n) {
    const double* al = ab + F1.aboff + (int64_t)j * 2 * m;
    const double* be = al + m;
    const double sa = ab[F1.sumoff + 2 * (int64_t)j], sb = ab[F1.sumoff + 2 * (int64_t)j + 1];
    for (int kk = lane; kk < m; kk += 64) {
      // row kk of F1^(j) and row j of F2^(kk) share the conservation row (j,kk)
      const double* al2 = ab + F2.aboff + (int64_t)kk * 2 * n;
      const double sb2 = ab[F2.sumoff + 2 * (int64_t)kk + 1];
      const double x1 = sg * (rowsum_prev[F1.rsoff + (int64_t)j * m + kk] -
                              (fam_cr(ab, F1, kk) - m * al[kk] - sb));
      const double x2 = sg * (rowsum_prev[F2.rsoff + (int64_t)kk * n + j] -
                              (fam_cr(ab, F2, j) - n * al2[j] - sb2));
      const double r = x1 - x2;
      prim += r * r;
    }
    const double* cpj = colpart_prev + F1.cpoff + (int64_t)j * F1.nchunk * m;
    for (int i = lane; i < m; i += 64) {
      double cs = 0.0;
      for (int c = 0; c < F1.nchunk; ++c) cs += cpj[(int64_t)c * m + i];
      const double x = sg * (cs - (fam_cr(ab, F1, i) - sa - m * be[i]));
      const double r = x - mu1T[(int64_t)j * m + i];
      prim += r * r;
      by += mu1T[(int64_t)j * m + i] * be[i];
    }
  }
  if (k < m) {
    const double* al = ab + F2.aboff + (int64_t)k * 2 * n;
    const double* be = al + n;
    const double sa = ab[F2.sumoff + 2 * (int64_t)k];
    const double* cpk = colpart_prev + F2.cpoff + (int64_t)k * F2.nchunk * n;
    for (int l = lane; l < n; l += 64) {
      if (k == m - 1 && l == n - 1) continue;
      double cs = 0.0;
      for (int c = 0; c < F2.nchunk; ++c) cs += cpk[(int64_t)c * n + l];
      const double x = sg * (cs - (fam_cr(ab, F2, l) - sa - n * be[l]));
      const double r = x - mu2[(int64_t)k * n + l];
      prim += r * r;
      by += mu2[(int64_t)k * n + l] * be[l];
    }
  }
  part[KP_PRIM] = prim;
  part[KP_BY] = by;
  __syncthreads();
  for (int q = 0; q < 8; ++q) {
    const double v = wave_sum(part[q]);
    if (lane == 0) wred[wave][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int q = threadIdx.x;
    vec[vec_kpart(G) + (int64_t)b * kKP + q] = (wred[0][q] + wred[1][q]) + (wred[2][q] + wred[3][q]);
  }
}

// ---------------------------------------------------------------------------
// Decision after a pass (taken by one wave of every solve block of the pair,
// on identical data, so all blocks agree).
// ---------------------------------------------------------------------------
// KKT partials of a pair reduced by one wave (fixed lane-strided order, then a
// butterfly); every lane returns the totals.
__device__ inline void reduce_kpart(const PairGeo& G, const double* vec, int lane, double* acc) {
  const double* kp = vec + vec_kpart(G);
  for (int q = 0; q < 8; ++q) {
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
//   kind 0, row block b: wave w writes beta of slab 4b + w (F1 slabs j
//           first, then F2 slabs k) and the slab's (sum alpha, sum beta);
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

template <int FROM_R>
__device__ inline double t_entry(const PairGeo& G, const double* vec, const double* ab,
                                 const SolveScalars& S,
                                 int k) {
  const double dm = (double)G.m;
  const double d = dinv(G.m, k);
  return (Sp_of<FROM_R>(G, vec, ab, k) - S.sa / dm) * d + dm * (dm + 1.0) * S.u * d;
}

// 1^T (Rhat1^j + Q t)
template <int FROM_R>
__device__ inline double rs_of(const PairGeo& G, const double* vec, const double* ab,
                               const SolveScalars& S, int j) {
  return b1_of<FROM_R>(G, vec, ab, j) - vec[vec_a(G) + j] + S.sp / (double)G.n + S.sq;
}

// beta of one slab, and the slab's (sum alpha, sum beta): sum_k y1[j][k] =
// rs_j / n and sum_j y1[j][k] = t[k] in closed form.
template <int FROM_R>
__device__ void solve_beta(const PairGeo& G, int slab, const double* arr, const double* vec,
                           double* ab, const SolveScalars& S, int lane) {
  const int m = G.m, n = G.n;
  const double dm = (double)m, dn = (double)n;
  if (slab < n) {  // F1^(j): beta = y2[j][.]
    const int j = slab;
    const double* R2 = arr + arr_R2(G);
    const FamGeo F = G.f[0];
    double* be = ab + F.aboff + (int64_t)j * 2 * m + m;
    const double rsj = rs_of<FROM_R>(G, vec, ab, S, j);
    double sb = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double v = (R2[(int64_t)j * m + i] - rsj / dn) / dm;
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
    const double tk = t_entry<FROM_R>(G, vec, ab, S, k);
    double sb = 0.0;
    for (int l = lane; l < n; l += 64) {
      const double v = (k == m - 1 && l == n - 1) ? 0.0 : (R3T[(int64_t)k * n + l] + tk) / dn;
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

// y1 on a 32 x 32 tile.  R1[j][k] comes from the two row-sum arrays (or is
// read directly for FROM_R).
template <int FROM_R>
__device__ void solve_alpha_tile(const PairGeo& G, int tile, const double* rowsum,
                                 const double* arr, const double* vec, double* ab,
                                 const SolveScalars& S) {
  __shared__ double T1[32][33], T2[32][33], Y[32][33];
  __shared__ double s_rs[32], s_a[32], s_cn[32], s_qt[32], s_p3[32], s_cm[32];
  const int m = G.m, n = G.n;
  const double dm = (double)m, dn = (double)n;
  const int jt = tile % G.ntj, kt = tile / G.ntj;
  const int j0 = 32 * jt, k0 = 32 * kt;
  const int t = threadIdx.x;
  const FamGeo F1 = G.f[0], F2 = G.f[1];
  if (t < 32) {
    const int j = j0 + t;
    if (j < n) {
      s_rs[t] = rs_of<FROM_R>(G, vec, ab, S, j);
      s_a[t] = vec[vec_a(G) + j];
      s_cn[t] = fam_cr(ab, F2, j);
    }
  } else if (t < 64) {
    const int kk = t - 32, k = k0 + kk;
    if (k < m) {
      const double tk = t_entry<FROM_R>(G, vec, ab, S, k);
      s_qt[kk] = (k == m - 1) ? tk - tk / dn : tk;
      s_p3[kk] = vec[vec_PR3(G) + k];
      s_cm[kk] = fam_cr(ab, F1, k);
    }
  }
  const double* rs1 = rowsum + F1.rsoff;  // [n][m]
  const double* rs2 = rowsum + F2.rsoff;  // [m][n]
  const double* R1 = arr + arr_R1(G);
  for (int e = t; e < 1024; e += kWG) {
    const int r = e >> 5, c = e & 31;
    const int j = j0 + r, k = k0 + c;        // T1[r][c] = (j, k)
    T1[r][c] = (j < n && k < m) ? (FROM_R ? R1[(int64_t)j * m + k] : rs1[(int64_t)j * m + k]) : 0.0;
    if (!FROM_R) {
      const int k2 = k0 + r, j2 = j0 + c;    // T2[r][c] = rs2[k2][j2]
      T2[r][c] = (k2 < m && j2 < n) ? rs2[(int64_t)k2 * n + j2] : 0.0;
    }
  }
  __syncthreads();
  for (int e = t; e < 1024; e += kWG) {
    const int jj = e >> 5, kk = e & 31;
    const int j = j0 + jj, k = k0 + kk;
    if (j < n && k < m) {
      const double r1 =
          FROM_R ? T1[jj][kk] : -(T1[jj][kk] - s_cm[kk]) + (T2[kk][jj] - s_cn[jj]);
      const double rh = r1 - s_a[jj] / dm + s_p3[kk] / dn;
      const double y = (rh + s_qt[kk] + s_rs[jj] / dn) / (dm + dn);
      ab[F1.aboff + (int64_t)j * 2 * m + k] = y;
      Y[jj][kk] = y;
    }
  }
  __syncthreads();
  for (int e = t; e < 1024; e += kWG) {
    const int kk = e >> 5, jj = e & 31;
    const int j = j0 + jj, k = k0 + kk;
    if (j < n && k < m) ab[F2.aboff + (int64_t)k * 2 * n + j] = -Y[jj][kk];
  }
}

template <int FROM_R>
__global__ __launch_bounds__(kWG) void k_pair_solve(const PBlock* __restrict__ sblocks,
                                                    const PairGeo* __restrict__ geo,
                                                    const PairCtl* __restrict__ ctl,
                                                    PairCtl* __restrict__ ctl_next,
                                                    const double* __restrict__ rowsum,
                                                    const double* __restrict__ arr,
                                                    const double* __restrict__ vec,
                                                    double* __restrict__ ab) {
  __shared__ PairCtl s_nx;
  __shared__ SolveScalars s_S;
  __shared__ int s_solve;
  const PBlock pbk = sblocks[blockIdx.x];
  const bool head = (pbk.kind == 0 && pbk.blk == 0 && threadIdx.x == 0);
  if (!FROM_R) {
    const PairCtl* cp = ctl + pbk.pair;
    if (cp->status != ST_RUNNING || cp->mode == MODE_IDLE) {
      if (head) ctl_next[pbk.pair] = *cp;
      return;
    }
  }
  const PairGeo G = geo[pbk.pair];
  if (threadIdx.x < 64) {  // wave 0 decides and rebuilds the solve scalars
    bool solve = true;
    PairCtl nx;
    if (!FROM_R) {
      const PairCtl c = ctl[pbk.pair];
      double acc[8];
      if (c.mode == MODE_CHECK) reduce_kpart(G, vec, threadIdx.x, acc);
      decide(G, c, acc, nx, solve);
    }
    SolveScalars S;
    if (solve) S = solve_scalars<FROM_R>(G, vec, ab, threadIdx.x);
    if (threadIdx.x == 0) {
      if (!FROM_R) s_nx = nx;
      s_solve = solve ? 1 : 0;
      if (solve) s_S = S;
    }
  }
  __syncthreads();
  if (s_solve) {
    if (pbk.kind == 0)
      solve_beta<FROM_R>(G, 4 * pbk.blk + (threadIdx.x >> 6), arr, vec, ab, s_S, threadIdx.x & 63);
    else
      solve_alpha_tile<FROM_R>(G, pbk.blk, rowsum, arr, vec, ab, s_S);
  }
  if (!FROM_R && head) ctl_next[pbk.pair] = s_nx;
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
  __shared__ double wred[4][4];
  const PBlock pbk = blocks[blockIdx.x];
  const PairGeo G = geo[pbk.pair];
  const int m = G.m, n = G.n, b = pbk.blk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (pbk.kind != 0) {  // strip slots carry no partial on this path
    if (pbk.kind == 1 && threadIdx.x < 4) vec[vec_spart(G) + 4 * (int64_t)(G.nblk + b) + threadIdx.x] = 0.0;
    return;
  }
  const double* R1 = arr + arr_R1(G);
  const double* R2 = arr + arr_R2(G);
  const double* R3T = arr + arr_R3T(G);
  const int j = 4 * b + wave, k = 4 * b + wave;
  double p_sa = 0.0, p_sp = 0.0, p_u = 0.0;
  if (j < n) {
    double s1 = 0.0, s2 = 0.0;
    for (int kk = lane; kk < m; kk += 64) s1 += R1[(int64_t)j * m + kk];
    for (int i = lane; i < m; i += 64) s2 += R2[(int64_t)j * m + i];
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      vec[vec_b1(G) + j] = s1;
      vec[vec_a(G) + j] = s2;
    }
    p_sa = s2;
  }
  if (k < m) {
    double s3 = 0.0, c1 = 0.0;
    for (int l = lane; l < n; l += 64) s3 += R3T[(int64_t)k * n + l];
    for (int jj = lane; jj < n; jj += 64) c1 += R1[(int64_t)jj * m + k];
    s3 = wave_sum(s3);
    c1 = wave_sum(c1);
    if (lane == 0) {
      vec[vec_PR3(G) + k] = s3;
      vec[vec_Sp(G) + k] = c1 + s3;
    }
    p_sp = s3;
    p_u = (c1 + s3) * dinv(m, k);
  }
  if (lane == 0) {
    wred[wave][0] = p_sa;
    wred[wave][1] = p_sp;
    wred[wave][2] = p_u;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int q = threadIdx.x;
    vec[vec_spart(G) + 4 * (int64_t)b + q] = (wred[0][q] + wred[1][q]) + (wred[2][q] + wred[3][q]);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage inside the library).
// ---------------------------------------------------------------------------


template <typename T, int V, int U, int C>
static void launch_lean(const LaunchArgs& a, int par, hipStream_t st) {
  hipLaunchKernelGGL((k_slab_pass<T, V, 0, U, C>), dim3(a.slab_grid), dim3(kWG), 0, st, a.items,
                     a.nitems, a.geo, a.ctl[par], (T*)a.sb[0], (T*)a.sb[1], (T*)a.sb[2], a.ab,
                     a.rowsum[par], a.colpart[par], a.kitem, a.bytes_ctr);
}

template <typename T, int V>
static void launch_slab(const LaunchArgs& a, int par, hipStream_t st) {
  if (a.coord) {  // non-uniform bins: positions from LDS, one row per wave step
    if (a.nt_store) launch_lean<T, V, 5, 1>(a, par, st);
    else launch_lean<T, V, 1, 1>(a, par, st);
    hipLaunchKernelGGL((k_slab_pass<T, V, 1, 1, 1>), dim3(a.slab_grid), dim3(kWG), 0, st, a.items,
                       a.nitems, a.geo, a.ctl[par], (T*)a.sb[0], (T*)a.sb[1], (T*)a.sb[2], a.ab,
                       a.rowsum[par], a.colpart[par], a.kitem, a.bytes_ctr);
    return;
  }
  const int u = (a.unroll >= 2 ? 2 : 1) | (a.nt_store ? 4 : 0);
  switch (u) {
    case 1: launch_lean<T, V, 1, 0>(a, par, st); break;
    case 2: launch_lean<T, V, 2, 0>(a, par, st); break;
    case 5: launch_lean<T, V, 5, 0>(a, par, st); break;
    default: launch_lean<T, V, 6, 0>(a, par, st); break;
  }
  hipLaunchKernelGGL((k_slab_pass<T, V, 1, 1, 0>), dim3(a.slab_grid), dim3(kWG), 0, st, a.items,
                     a.nitems, a.geo,
                     a.ctl[par], (T*)a.sb[0], (T*)a.sb[1], (T*)a.sb[2], a.ab, a.rowsum[par],
                     a.colpart[par], a.kitem, a.bytes_ctr);
}

template <typename T>
static void launch_slab_t(const LaunchArgs& a, int par, hipStream_t st) {
  if (a.maxvpl <= 1) launch_slab<T, 1>(a, par, st);
  else if (a.maxvpl <= 2) launch_slab<T, 2>(a, par, st);
  else if (a.maxvpl <= 4) launch_slab<T, 4>(a, par, st);
  else launch_slab<T, 8>(a, par, st);
}

void launch_slab_pass(const LaunchArgs& a, int par, hipStream_t st) {
  if (a.fp32) launch_slab_t<float>(a, par, st);
  else launch_slab_t<double>(a, par, st);
}

void launch_pair_kernels(const LaunchArgs& a, int par, hipStream_t st) {
  hipLaunchKernelGGL(k_pair_reduce, dim3(a.nblocks), dim3(kWG), 0, st, a.blocks, a.geo,
                     a.ctl[par], a.rowsum[par], a.colpart[par], a.rowsum[1 - par],
                     a.colpart[1 - par], a.kitem, a.ab, a.arr, a.vec);
  hipLaunchKernelGGL(k_pair_solve<0>, dim3(a.nsblocks), dim3(kWG), 0, st, a.sblocks, a.geo,
                     a.ctl[par], a.ctl[1 - par], (const double*)a.rowsum[par], a.arr, a.vec, a.ab);
}

// One iteration: slab pass, pair reduce, pair solve.  Reads ctl[par], writes ctl[1-par].
void launch_iteration(const LaunchArgs& a, int par, hipStream_t st) {
  launch_slab_pass(a, par, st);
  hipLaunchKernelGGL(k_pair_reduce, dim3(a.nblocks), dim3(kWG), 0, st, a.blocks, a.geo,
                     a.ctl[par], a.rowsum[par], a.colpart[par], a.rowsum[1 - par],
                     a.colpart[1 - par], a.kitem, a.ab, a.arr, a.vec);
  hipLaunchKernelGGL(k_pair_solve<0>, dim3(a.nsblocks), dim3(kWG), 0, st, a.sblocks, a.geo,
                     a.ctl[par], a.ctl[1 - par], (const double*)a.rowsum[par], a.arr, a.vec, a.ab);
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
  hipLaunchKernelGGL(k_pair_solve<1>, dim3(a.nsblocks), dim3(kWG), 0, st, a.sblocks, a.geo,
                     (const PairCtl*)nullptr, (PairCtl*)nullptr, (const double*)nullptr, a.arr,
                     a.vec, a.ab);
}

}  // namespace hot

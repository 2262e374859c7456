// Slab pass of the HOT iteration (arXiv 2408.00598, Algorithm 2, Steps 2-4
// fused with the sums Step 1 of the next iteration needs) for gfx950: streams
// every slab of the flow state once, computes g = c - A^T ybar,
// shat = |s - 2g| and the Halpern step, writes the new state and its row /
// column sums, and on check passes the partial sums of the relative KKT
// residual (eq. kkt_res).  This is the bandwidth-bound kernel of the path.
#include "hot_device.h"
#include "hot_internal.h"
#include "hot_runtime.h"

namespace hot {

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
  double sig_old, ratio;  // sigma re-balancing at a restart: x_bar's sigma, old/new
};

// SU = 1 (check and restart passes of a problem with sigma re-balancing):
// check passes also read x_bar of the last restart (xr) and accumulate
// ||x_bar - X||^2; restart passes write x_bar to xr and the new state
// x_bar / sigma_new + z_bar = (sigma_old / sigma_new)(s - g) + max(0, 2g - s).
template <typename T, int MAXVPL, int MODE, int ANC, int U, int C, int SU>
__device__ __forceinline__ void slab_rows(const SlabCtx& x, const T* __restrict__ src,
                                 T* __restrict__ dst, const T* __restrict__ anc,
                                 T* __restrict__ xr,
                                 const double* __restrict__ alpha, const double* __restrict__ bl,
                                 const double* __restrict__ lx,
                                 double (&colacc)[MAXVPL][VecT<T>::W], double* __restrict__ rowsum,
                                 double (&kk)[7]) {
  constexpr int W = VecT<T>::W;
  typedef typename VecT<T>::type VT;
  constexpr bool RDX = SU && MODE == MODE_CHECK;    // read X
  constexpr bool WRX = SU && MODE == MODE_RESTART;  // write X
  const int LR = 1 << x.lrs, rpw = 64 >> x.lrs;
  const int L = x.L, P = x.P;
  constexpr int UR = U & 3;
  for (int pb = x.r0 + x.wave * rpw; pb < x.r1; pb += 4 * UR * rpw) {
    int prow[UR];
    bool rvv[UR];
    VT xs[UR][MAXVPL], xa[UR][MAXVPL];
    VT xq[RDX ? UR : 1][RDX ? MAXVPL : 1];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      prow[u] = pb + u * 4 * rpw + x.slot;
      rvv[u] = prow[u] < x.r1;
#pragma unroll
      for (int v = 0; v < MAXVPL; ++v) {
        const int q0 = (x.lin + (v << x.lrs)) * W;
        if (v < x.vpl && rvv[u] && q0 < L) {
          xs[u][v] = vload_nt<T>(src + (int64_t)prow[u] * P + q0);
          if (ANC == ANC_SEP) xa[u][v] = vload_nt<T>(anc + (int64_t)prow[u] * P + q0);
          if constexpr (RDX) xq[u][v] = vload_nt<T>(xr + (int64_t)prow[u] * P + q0);
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
          VT out, outx;
          const double d0 = (double)(p - q0);
#pragma unroll
          for (int e = 0; e < W; ++e) {
            const bool ok = (q0 + e) < L;
            const double s = (double)vget(xs[u][v], e);
            const double d = C ? xp - lx[q0 + e] : d0 - (double)e;
            const double g = d * d - (ap + bl[q0 + e]);
            double o;
            if (MODE == MODE_RESTART) {
              if constexpr (WRX) {
                const double dd = s - g;
                o = x.ratio * dd + fmax(0.0, 2.0 * g - s);
                vset(outx, e, ok ? (T)(x.sig_old * dd) : (T)0);
              } else {
                o = fmax(s - g, g);
              }
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
                if constexpr (RDX) {
                  const double dxe = xb - (double)vget(xq[u][v], e);
                  kk[KI_DX] += ok ? dxe * dxe : 0.0;
                }
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
          if constexpr (WRX) *reinterpret_cast<VT*>(xr + (int64_t)p * P + q0) = outx;
        }
      }
      rowacc = group_sum(rowacc, LR);
      if (rv && x.lin == LR - 1) rowsum[p] = rowacc;
    }
  }
}

// HEAVY = 0: plain update passes; HEAVY = 1: check and restart passes (when
// both are launched every iteration, a workgroup whose pair is in the other
// kind of pass exits at once).  HEAVY = 2: every pass kind in one kernel,
// check and restart rows streamed one row step at a time as in HEAVY = 1;
// on uniform bins its register count stays that of the plain kernel, and the
// launch it saves is worth 2-6% of a solve.  The three are forced inline into their kernels:
// a second caller would otherwise turn slab_item into a real call, which
// more than doubles the register count.
template <typename T, int MAXVPL, int HEAVY, int U, int C, int SU>
__device__ __forceinline__ void slab_item(
    int item, const SlabItem* __restrict__ items, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, T* __restrict__ sb0, T* __restrict__ sb1,
    T* __restrict__ sb2, T* __restrict__ sbx, const double* __restrict__ ab,
    double* __restrict__ rowsum,
    double* __restrict__ colpart, double* __restrict__ kitem,
    double* lds_col, double* lds_beta, double* lds_x, double* red) {
  constexpr int W = VecT<T>::W;
  constexpr int S = 64 * MAXVPL * W;
  const SlabItem itm = items[item];
  const PairCtl* cp = ctl + itm.pair;
  const int status = cp->status;
  const int mode = cp->mode;
  if (status != ST_RUNNING) return;
  if (HEAVY == 0 && mode != MODE_NORMAL) return;
  if (HEAVY == 1 && mode != MODE_CHECK && mode != MODE_RESTART) return;
  if (mode != MODE_NORMAL && mode != MODE_CHECK && mode != MODE_RESTART) return;
  const bool plain = mode == MODE_NORMAL;
  if (plain && itm.small) return;  // (the wave-per-slab kernel runs these)
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
  x.sig_old = cp->sig_old;
  x.ratio = cp->sig_old / cp->sigma;
  // (SU kernels only) this problem re-balances sigma at restarts
  const bool su = SU && HEAVY && (cp->flags & 0x10) != 0;
  const int L = F.L;
  const int64_t soff = F.soff + (int64_t)itm.slab * L * F.P;
  const int src_i = cp->src, anc_i = cp->anc;
  const int dst_i = (mode == MODE_RESTART) ? 2 : cp->dst;
  const T* src = pick<T>(sb0, sb1, sb2, src_i) + soff;
  T* dst = pick<T>(sb0, sb1, sb2, dst_i) + soff;
  const int anc_kind =
      (mode == MODE_RESTART || anc_i < 0) ? ANC_ZERO : (anc_i == src_i ? ANC_SAME : ANC_SEP);
  const T* anc = anc_kind == ANC_SEP ? pick<T>(sb0, sb1, sb2, anc_i) + soff : src;
  T* xr = su ? sbx + soff : nullptr;
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
  double kk[7] = {0, 0, 0, 0, 0, 0, 0};
  // check and restart rows: one row step at a time; plain rows: the
  // launch's unroll and store kind
  constexpr int UH = HEAVY == 2 ? 1 : U;
#define HOT_ROWS(MODE_, ANC_, SU_)                                                        \
  slab_rows<T, MAXVPL, MODE_, ANC_, (MODE_ == MODE_NORMAL ? U : UH), C, SU_>(             \
      x, src, dst, anc, xr, alpha, lds_beta, lds_x, colacc, rs, kk)
  if (HEAVY != 1 && plain) {
    if (anc_kind == ANC_ZERO) HOT_ROWS(MODE_NORMAL, ANC_ZERO, 0);
    else if (anc_kind == ANC_SAME) HOT_ROWS(MODE_NORMAL, ANC_SAME, 0);
    else HOT_ROWS(MODE_NORMAL, ANC_SEP, 0);
  } else if (HEAVY == 0) {
    // (not reached: the mode test above; keeps the check and restart code
    // out of the plain kernel)
  } else if (mode == MODE_CHECK) {
    bool done = false;
    if constexpr (SU) {
      if (su) {
        if (anc_kind == ANC_ZERO) HOT_ROWS(MODE_CHECK, ANC_ZERO, 1);
        else if (anc_kind == ANC_SAME) HOT_ROWS(MODE_CHECK, ANC_SAME, 1);
        else HOT_ROWS(MODE_CHECK, ANC_SEP, 1);
        done = true;
      }
    }
    if (!done) {
      if (anc_kind == ANC_ZERO) HOT_ROWS(MODE_CHECK, ANC_ZERO, 0);
      else if (anc_kind == ANC_SAME) HOT_ROWS(MODE_CHECK, ANC_SAME, 0);
      else HOT_ROWS(MODE_CHECK, ANC_SEP, 0);
    }
  } else {
    bool done = false;
    if constexpr (SU) {
      if (su) {
        HOT_ROWS(MODE_RESTART, ANC_ZERO, 1);
        done = true;
      }
    }
    if (!done) HOT_ROWS(MODE_RESTART, ANC_ZERO, 0);
  }
#undef HOT_ROWS

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
  if (HEAVY && mode == MODE_CHECK) {
    // all partials at once: wave sums, one barrier, then the fixed order
    // (w0 + w1) + (w2 + w3) per partial
    double* ko = kitem + (int64_t)itm.kslot * kKI;
    const int nq = su ? 7 : 6;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const double v = wave_sum(kk[q]);
      if (q < nq && x.lane == 0) red[x.wave * 8 + q] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nq) {
      const int q = threadIdx.x;
      ko[q] = (red[q] + red[8 + q]) + (red[16 + q] + red[24 + q]);
    }
  }
}

// One workgroup per item.  SU = 1 (check / restart kernel only): some problem
// of the launch re-balances sigma at restarts.
template <typename T, int MAXVPL, int HEAVY, int U, int C, int SU>
__global__ __launch_bounds__(kWG) void k_slab_pass(
    const SlabItem* __restrict__ items, int nitems, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, T* __restrict__ sb0, T* __restrict__ sb1,
    T* __restrict__ sb2, T* __restrict__ sbx, const double* __restrict__ ab,
    double* __restrict__ rowsum,
    double* __restrict__ colpart, double* __restrict__ kitem) {
  constexpr int W = VecT<T>::W;
  constexpr int S = 64 * MAXVPL * W;
  __shared__ double lds_col[4 * S];
  __shared__ double lds_beta[S];
  __shared__ double lds_x[C ? S : 1];
  __shared__ double red[32];
  if ((int)blockIdx.x < nitems)
    slab_item<T, MAXVPL, HEAVY, U, C, SU>(blockIdx.x, items, geo, ctl, sb0, sb1, sb2, sbx, ab, rowsum,
                                      colpart, kitem, lds_col, lds_beta, lds_x, red);
}

// ---------------------------------------------------------------------------
// Wave-per-slab plain-update pass for small slabs (side <= a tunable, 48 by
// default).  A block pass over a 32 x 32 slab keeps most of a workgroup idle
// and pays two barriers and an LDS round trip for 4 KB of state; here each
// wave owns a whole slab: beta (and the column positions) sit in registers
// for the lane's fixed columns, rows are streamed in steps of 64 / LR, the row
// sums use the same DPP tree and the column sums fold the wave's row slots
// with shuffles, so the kernel has no barrier at all.  The arithmetic per
// element is the block pass's, term for term.
// ---------------------------------------------------------------------------
template <typename T, int MAXVPL, int ANC, int U, int C>
__device__ __forceinline__ void slab_wave(const SlabCtx& x, const T* __restrict__ src,
                                 T* __restrict__ dst, const T* __restrict__ anc,
                                 const double* __restrict__ alpha,
                                 const double* __restrict__ beta, const double* __restrict__ X,
                                 double* __restrict__ rowsum, double* __restrict__ colout) {
  constexpr int W = VecT<T>::W;
  typedef typename VecT<T>::type VT;
  const int LR = 1 << x.lrs, rpw = 64 >> x.lrs;
  const int L = x.L, P = x.P;
  constexpr int UR = U & 3;
  double bq[MAXVPL][W], xq[C ? MAXVPL : 1][C ? W : 1], colacc[MAXVPL][W];
#pragma unroll
  for (int v = 0; v < MAXVPL; ++v)
#pragma unroll
    for (int e = 0; e < W; ++e) {
      const int q = (x.lin + (v << x.lrs)) * W + e;
      const bool in = v < x.vpl && q < L;
      bq[v][e] = in ? beta[q] : 0.0;
      if constexpr (C) xq[v][e] = in ? X[q] : 0.0;
      colacc[v][e] = 0.0;
    }
  for (int pb = x.slot; pb < L; pb += UR * rpw) {
    int prow[UR];
    bool rvv[UR];
    VT xs[UR][MAXVPL], xa[UR][MAXVPL];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      prow[u] = pb + u * rpw;
      rvv[u] = prow[u] < L;
#pragma unroll
      for (int v = 0; v < MAXVPL; ++v) {
        const int q0 = (x.lin + (v << x.lrs)) * W;
        if (v < x.vpl && rvv[u] && q0 < L) {
          xs[u][v] = vload_nt<T>(src + (int64_t)prow[u] * P + q0);
          if (ANC == ANC_SEP) xa[u][v] = vload_nt<T>(anc + (int64_t)prow[u] * P + q0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int p = prow[u];
      const bool rv = rvv[u];
      const double ap = rv ? alpha[p] : 0.0;
      const double xp = (C && rv) ? X[p] : 0.0;
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
            double d;
            if constexpr (C) d = xp - xq[v][e];
            else d = d0 - (double)e;
            const double g = d * d - (ap + bq[v][e]);
            const double sh = fabs(s - 2.0 * g);
            double o;
            if (ANC == ANC_ZERO) o = x.oml * sh;
            else if (ANC == ANC_SAME) o = x.lam * s + x.oml * sh;
            else o = x.lam * (double)vget(xa[u][v], e) + x.oml * sh;
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
  // column sums: fold the wave's row slots
#pragma unroll
  for (int v = 0; v < MAXVPL; ++v)
#pragma unroll
    for (int e = 0; e < W; ++e) {
      double t = colacc[v][e];
      for (int off = LR; off < 64; off <<= 1) t += __shfl_xor(t, off, 64);
      const int q = (x.lin + (v << x.lrs)) * W + e;
      if (x.slot == 0 && v < x.vpl && q < L) colout[q] = t;
    }
}

template <typename T, int MAXVPL, int U, int C>
__global__ __launch_bounds__(kWG) void k_slab_small(
    const SmallItem* __restrict__ items, const PairGeo* __restrict__ geo,
    const PairCtl* __restrict__ ctl, T* __restrict__ sb0, T* __restrict__ sb1,
    T* __restrict__ sb2, const double* __restrict__ ab, double* __restrict__ rowsum,
    double* __restrict__ colpart) {
  const SmallItem itm = items[blockIdx.x];
  const int wave = threadIdx.x >> 6;
  if (wave >= itm.nslab) return;
  const PairCtl* cp = ctl + itm.pair;
  if (cp->status != ST_RUNNING || cp->mode != MODE_NORMAL) return;
  const FamGeo F = geo[itm.pair].f[itm.fam];
  const int slab = itm.slab0 + wave;
  SlabCtx x;
  x.L = F.L;
  x.P = F.P;
  x.r0 = 0;
  x.r1 = F.L;
  x.lrs = F.lrs;
  x.vpl = F.vpl;
  x.lane = threadIdx.x & 63;
  x.wave = wave;
  x.slot = x.lane >> x.lrs;
  x.lin = x.lane & ((1 << x.lrs) - 1);
  x.lam = cp->lam;
  x.oml = 1.0 - cp->lam;
  x.sigma = cp->sigma;
  const int L = F.L;
  const int64_t soff = F.soff + (int64_t)slab * L * F.P;
  const int src_i = cp->src, anc_i = cp->anc;
  const T* src = pick<T>(sb0, sb1, sb2, src_i) + soff;
  T* dst = pick<T>(sb0, sb1, sb2, cp->dst) + soff;
  const int anc_kind = anc_i < 0 ? ANC_ZERO : (anc_i == src_i ? ANC_SAME : ANC_SEP);
  const T* anc = anc_kind == ANC_SEP ? pick<T>(sb0, sb1, sb2, anc_i) + soff : src;
  const double* alpha = ab + F.aboff + (int64_t)slab * 2 * L;
  const double* X = fam_x(ab, F);
  double* rs = rowsum + F.rsoff + (int64_t)slab * L;
  double* co = colpart + F.cpoff + (int64_t)slab * F.nchunk * L;  // one chunk
  if (anc_kind == ANC_ZERO)
    slab_wave<T, MAXVPL, ANC_ZERO, U, C>(x, src, dst, anc, alpha, alpha + L, X, rs, co);
  else if (anc_kind == ANC_SAME)
    slab_wave<T, MAXVPL, ANC_SAME, U, C>(x, src, dst, anc, alpha, alpha + L, X, rs, co);
  else
    slab_wave<T, MAXVPL, ANC_SEP, U, C>(x, src, dst, anc, alpha, alpha + L, X, rs, co);
}

template <typename T, int V, int U, int C>
static void launch_lean(const LaunchArgs& a, int par, hipStream_t st) {
  if (a.nbig > 0)
    hipLaunchKernelGGL((k_slab_pass<T, V, 0, U, C, 0>), dim3(a.nbig), dim3(kWG), 0, st,
                       a.items, a.nbig, a.geo, a.ctl[par], (T*)a.sb[0], (T*)a.sb[1],
                       (T*)a.sb[2], (T*)a.sbx, a.ab, a.rowsum[par], a.colpart[par], a.kitem);
  if (a.nsitems > 0)
    hipLaunchKernelGGL((k_slab_small<T, V, (U & 4) | 2, C>), dim3(a.nsitems), dim3(kWG), 0, st,
                       a.sitems, a.geo, a.ctl[par], (T*)a.sb[0], (T*)a.sb[1], (T*)a.sb[2], a.ab,
                       a.rowsum[par], a.colpart[par]);
}

template <typename T, int V, int C, int SU>
static void launch_heavy(const LaunchArgs& a, int par, hipStream_t st) {
  hipLaunchKernelGGL((k_slab_pass<T, V, 1, 1, C, SU>), dim3(a.nitems), dim3(kWG), 0, st,
                     a.items, a.nitems, a.geo, a.ctl[par], (T*)a.sb[0], (T*)a.sb[1],
                     (T*)a.sb[2], (T*)a.sbx, a.ab, a.rowsum[par], a.colpart[par], a.kitem);
}

// Every pass of the block items in one kernel (plain, check, restart), plus
// the wave-per-slab kernel for small slabs.
template <typename T, int V, int U, int C, int SU>
static void launch_fused(const LaunchArgs& a, int par, hipStream_t st) {
  hipLaunchKernelGGL((k_slab_pass<T, V, 2, U, C, SU>), dim3(a.nitems), dim3(kWG), 0, st,
                     a.items, a.nitems, a.geo, a.ctl[par], (T*)a.sb[0], (T*)a.sb[1],
                     (T*)a.sb[2], (T*)a.sbx, a.ab, a.rowsum[par], a.colpart[par], a.kitem);
  if (a.nsitems > 0)
    hipLaunchKernelGGL((k_slab_small<T, V, (U & 4) | 2, C>), dim3(a.nsitems), dim3(kWG), 0, st,
                       a.sitems, a.geo, a.ctl[par], (T*)a.sb[0], (T*)a.sb[1], (T*)a.sb[2], a.ab,
                       a.rowsum[par], a.colpart[par]);
}

template <typename T, int V>
static void launch_slab(const LaunchArgs& a, int par, hipStream_t st) {
  if (a.fuse && a.coord) {  // non-uniform bins: one row per wave step
    if (a.nt_store) {
      if (a.su) launch_fused<T, V, 5, 1, 1>(a, par, st);
      else launch_fused<T, V, 5, 1, 0>(a, par, st);
    } else {
      if (a.su) launch_fused<T, V, 1, 1, 1>(a, par, st);
      else launch_fused<T, V, 1, 1, 0>(a, par, st);
    }
    return;
  }
  if (a.fuse) {
    const int u = (a.unroll >= 2 ? 2 : 1) | (a.nt_store ? 4 : 0);
    if (a.su) {
      switch (u) {
        case 1: launch_fused<T, V, 1, 0, 1>(a, par, st); break;
        case 2: launch_fused<T, V, 2, 0, 1>(a, par, st); break;
        case 5: launch_fused<T, V, 5, 0, 1>(a, par, st); break;
        default: launch_fused<T, V, 6, 0, 1>(a, par, st); break;
      }
    } else {
      switch (u) {
        case 1: launch_fused<T, V, 1, 0, 0>(a, par, st); break;
        case 2: launch_fused<T, V, 2, 0, 0>(a, par, st); break;
        case 5: launch_fused<T, V, 5, 0, 0>(a, par, st); break;
        default: launch_fused<T, V, 6, 0, 0>(a, par, st); break;
      }
    }
    return;
  }
  if (a.coord) {  // non-uniform bins: positions from LDS, one row per wave step
    if (a.nt_store) launch_lean<T, V, 5, 1>(a, par, st);
    else launch_lean<T, V, 1, 1>(a, par, st);
    if (a.su) launch_heavy<T, V, 1, 1>(a, par, st);
    else launch_heavy<T, V, 1, 0>(a, par, st);
    return;
  }
  const int u = (a.unroll >= 2 ? 2 : 1) | (a.nt_store ? 4 : 0);
  switch (u) {
    case 1: launch_lean<T, V, 1, 0>(a, par, st); break;
    case 2: launch_lean<T, V, 2, 0>(a, par, st); break;
    case 5: launch_lean<T, V, 5, 0>(a, par, st); break;
    default: launch_lean<T, V, 6, 0>(a, par, st); break;
  }
  if (a.su) launch_heavy<T, V, 0, 1>(a, par, st);
  else launch_heavy<T, V, 0, 0>(a, par, st);
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

}  // namespace hot

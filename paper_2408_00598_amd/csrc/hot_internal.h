// Internal data layout of libhot (not part of the C ABI).
//
// Storage of the flow state ("slab form" of the reduced model, Sec. 2.1):
//   family 0 (f1): n slabs F1^(j), each m x m, F1^(j)[k][i] = f1_{i,k,j};
//   family 1 (f2): m slabs F2^(k), each n x n, F2^(k)[j][l] = f2_{k,j,l}.
// Each slab is row-major with a row pitch P >= L (P a multiple of the 16-byte
// vector width); padding entries hold zero.  On a slab of side L the cost is
// C[p][q] = (p - q)^2 for both families, and A^T y restricted to the slab is
// alpha[p] + beta[q] with
//   F1^(j): alpha = y1[j][.] (row index k), beta = y2[j][.] (column index i);
//   F2^(k): alpha = -y1[.][k] (row index j), beta = y3[.][k] (column index l),
// so A x is made of the row and column sums of the slabs.
//
// The iteration is kept in the single-vector form s = x/sigma + z (the
// shadow sequence of the appendix, u = C^T w, scaled by 1/sqrt(sigma)):
//   R = b/sigma - A(s - c),  A A^T ybar = R,  g = c - A^T ybar,
//   xbar = sigma (s - g),  zbar = max(0, 2g - s),  shat = |s - 2g|,
//   s <- lam s0 + (1 - lam) shat,  lam = 1/(k+2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hot {

constexpr int kWG = 256;        // threads per workgroup of every kernel
constexpr int kKI = 8;          // per-item KKT partials written by the slab pass
constexpr int kKP = 12;         // per-block partials written by the pair reduce
constexpr int kMaxSide = 1024;  // largest supported m or n
constexpr int kWideSide = 256;  // slab side from which the pair reduce gives a
                                // slab a whole workgroup instead of one wave
constexpr int kMinSmallSlabs = 1024;  // fewest small slabs for the wave-per-slab pass

enum Mode : int32_t {
  MODE_IDLE = 0,
  MODE_NORMAL = 1,   // plain update pass
  MODE_CHECK = 2,    // update pass + KKT / fixed-point partials of w_bar^k
  MODE_RESTART = 3,  // write sbar = max(s - g, g) into the anchor buffer
  MODE_INIT = 4      // s = 0: only the first linear solve runs
};

enum PairStatus : int32_t {
  ST_RUNNING = 0,
  ST_CONVERGED = 1,
  ST_MAXITER = 2,
  ST_NUMERIC = 3,
  ST_FIXED_DONE = 4,
  ST_SYNC_LOST = 5  // fused reduce + solve: a wait ran out (device error)
};

// per-item partial indices (slab pass, check mode)
// (after the solve, the finalize pass reuses slots KI_DX and KI_NEG for
// ||x_bar||^2 and ||min(x_bar, 0)||^2 of the final iterate)
enum KItem : int { KI_DUAL = 0, KI_COMP, KI_XX, KI_ZZ, KI_CX, KI_FP, KI_DX, KI_NEG };
// per-block partial indices (pair reduce, check mode)
enum KPart : int { KP_DUAL = 0, KP_COMP, KP_XX, KP_ZZ, KP_CX, KP_FP, KP_DX, KP_PRIM, KP_BY, KP_DY };
constexpr int kNKP = 10;  // partials per reduce block in use (of kKP slots)

struct FamGeo {
  int32_t L;       // slab side
  int32_t P;       // row pitch in elements
  int32_t nslab;   // slabs in the family
  int32_t nchunk;  // row chunks per slab (one slab-pass item each)
  int32_t rpc;     // rows per chunk
  int32_t lrs;     // log2(lanes per row)
  int32_t vpl;     // 16-byte vectors per lane per row
  int32_t wide;    // 1: the pair reduce gives each slab a whole workgroup (its
                   // columns split over the four waves); 0: one wave per slab
  int64_t soff;    // element offset of slab 0 in each state buffer
  int64_t aboff;   // double offset of slab 0's alpha; beta follows (2L per slab)
  int64_t rsoff;   // double offset of the row sums (L per slab)
  int64_t cpoff;   // double offset of the column partials (nchunk*L per slab)
  int64_t sumoff;  // double offset of (sum alpha, sum beta) per slab (2 per slab)
  int64_t xoff;    // double offset of the family's cost table in the alpha/beta
                   // array: X[L] grid-line positions, CR[L] = sum_q (X_p - X_q)^2,
                   // then CC = sum_p CR[p]
};

// cost table of a family (written at set-up, read-only afterwards)
__host__ __device__ inline const double* fam_x(const double* ab, const FamGeo& F) { return ab + F.xoff; }
__host__ __device__ inline double fam_cr(const double* ab, const FamGeo& F, int p) {
  return ab[F.xoff + F.L + p];
}
__host__ __device__ inline double fam_cc(const double* ab, const FamGeo& F) {
  return ab[F.xoff + 2 * (int64_t)F.L];
}

struct PairGeo {
  int32_t m, n;
  int32_t item0, nitem;  // slab-pass items of this pair
  int32_t blk0, nblk;    // reduce slots of this pair: nb1 of F1 rows j, then F2 rows k
                         // (4 rows each, or 1 for a wide family; one KKT / solve-sum
                         // partial each); a reduce row block takes rq slots
  int32_t ns1, ns2;      // reduce strip blocks: 64 columns k of rs1 / 64 columns j of rs2
  int32_t sblk0, nsblk;  // solve row blocks (4 spw slabs each)
  int32_t ntj, ntk;      // solve tiles: 32 j x 32 k each
  int32_t ipb, nb1;      // slab items per reduce row block (KKT reduction); F1 row blocks
  int32_t spw, rq;       // slabs per wave of a solve row block (4 spw slabs per block);
                         // reduce slots per reduce row block of a narrow family
  FamGeo f[2];
  int64_t moff;          // double offset of the M-sized arrays (5 of them)
  int64_t voff;          // double offset of the small vectors
  double norm_b, norm_c; // ||b||, ||c|| of the reduced model
};

// Reduce and solve workgroups of a pair: the tables list every one of a
// running pair (the fused reduce + solve counts them).
__host__ __device__ inline int reduce_blocks_of(const PairGeo& G) {
  const int rq1 = G.f[0].wide ? 1 : G.rq, rq2 = G.f[1].wide ? 1 : G.rq;
  return (G.nb1 + rq1 - 1) / rq1 + (G.nblk - G.nb1 + rq2 - 1) / rq2 + G.ns1 + G.ns2;
}
__host__ __device__ inline int solve_blocks_of(const PairGeo& G) {
  return G.nsblk + G.ntj * G.ntk;
}

// M-sized arrays at moff: mu1T[j][i], mu2[k][l], R1[j][k], R2[j][i], R3T[k][l]
__host__ __device__ inline int64_t arr_mu1T(const PairGeo& g) { return g.moff; }
__host__ __device__ inline int64_t arr_mu2(const PairGeo& g) { return g.moff + (int64_t)g.m * g.n; }
__host__ __device__ inline int64_t arr_R1(const PairGeo& g) { return g.moff + 2 * (int64_t)g.m * g.n; }
__host__ __device__ inline int64_t arr_R2(const PairGeo& g) { return g.moff + 3 * (int64_t)g.m * g.n; }
__host__ __device__ inline int64_t arr_R3T(const PairGeo& g) { return g.moff + 4 * (int64_t)g.m * g.n; }
// small vectors at voff (per pair):
//   a[n]    row totals of R2 (a_j = 1^T R2^j)
//   tot1[n] row totals of the F1 row sums (sum_k rs1[j][k])
//   u2[n]   column totals of the F2 row sums (sum_k rs2[k][j])
//   b1[n]   1^T R1^j when R is given directly (Prop. 3 entry point)
//   PR3[m]  row totals of R3^T,  tot2[m] sum_j rs2[k][j],  u1[m] sum_j rs1[j][k]
//   Sp[m]   sum_j R1[j][k] + PR3[k] when R is given directly
//   spart[nblk + ns1][4]  per-block partials of (sum a_j, sum PR3, sum Sp/D)
//   kpart[nblk][kKP]      per-block KKT partials
__host__ __device__ inline int64_t vec_a(const PairGeo& g) { return g.voff; }
__host__ __device__ inline int64_t vec_tot1(const PairGeo& g) { return g.voff + (int64_t)g.n; }
__host__ __device__ inline int64_t vec_u2(const PairGeo& g) { return g.voff + 2 * (int64_t)g.n; }
__host__ __device__ inline int64_t vec_b1(const PairGeo& g) { return g.voff + 3 * (int64_t)g.n; }
__host__ __device__ inline int64_t vec_PR3(const PairGeo& g) { return g.voff + 4 * (int64_t)g.n; }
__host__ __device__ inline int64_t vec_tot2(const PairGeo& g) { return vec_PR3(g) + g.m; }
__host__ __device__ inline int64_t vec_u1(const PairGeo& g) { return vec_PR3(g) + 2 * (int64_t)g.m; }
__host__ __device__ inline int64_t vec_Sp(const PairGeo& g) { return vec_PR3(g) + 3 * (int64_t)g.m; }
__host__ __device__ inline int64_t vec_spart(const PairGeo& g) { return vec_PR3(g) + 4 * (int64_t)g.m; }
__host__ __device__ inline int64_t vec_kpart(const PairGeo& g) {
  return vec_spart(g) + 4 * (int64_t)(g.nblk + g.ns1);
}
__host__ __device__ inline int64_t vec_size(const PairGeo& g) {
  return 4 * (int64_t)g.n + 4 * (int64_t)g.m + 4 * (int64_t)(g.nblk + g.ns1) +
         (int64_t)g.nblk * kKP;
}

// One workgroup of the block slab pass: a row chunk of one slab.  kslot is
// the item's KKT-partial slot (contiguous per pair, in (fam, slab, chunk)
// order); small = 1 marks slabs whose plain-update passes run in the
// wave-per-slab kernel instead (the block kernels still run their check and
// restart passes).
struct SlabItem {
  int32_t pair, fam, slab, chunk;
  int32_t kslot, small, pad0, pad1;
};

// One workgroup of the wave-per-slab pass: up to four consecutive slabs of
// one family, one wave each (small slabs, whole slab per wave).
struct SmallItem {
  int32_t pair, fam, slab0, nslab;
};

struct PBlock {
  int32_t pair, blk, kind, pad;  // kind: see k_pair_reduce / k_pair_solve
};

struct PairCtl {
  double sigma, lam, tol;
  double r_start, r_prev;
  double kkt, res_p, res_d, res_c, pobj, dobj, fp_res;
  double kkt_abs, relax;  // ||R(w_bar)||; rho of the ADMM baseline (0: Halpern)
  double feaserr;         // max(||min(x_bar, 0)|| / (1 + ||x_bar||), res_p)
  double sig_old;         // restart pass with sigma re-balancing: sigma of x_bar
  int32_t k, it, restarts, status;
  int32_t mode, src, dst, anc;
  int32_t max_iter, T, flags, pad;
};

// closed form of sum_{q=0}^{L-1} (p - q)^2 (exact in FP64 for L <= 2^17)
__host__ __device__ inline double cost_rowsum(int L, int p) {
  const double dL = (double)L, dp = (double)p;
  const double s1 = dL * (dL - 1.0) * 0.5;
  const double s2 = (dL - 1.0) * dL * (2.0 * dL - 1.0) / 6.0;
  return dL * dp * dp - 2.0 * dp * s1 + s2;
}

}  // namespace hot

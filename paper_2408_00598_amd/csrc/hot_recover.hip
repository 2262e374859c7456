// Transport-plan recovery (Algorithm 1, alg:transportplan) and marginal
// repair on the device.
//
// For every bin (k,j), Algorithm 1 matches the flows entering the bin along
// its column, f1_{i,k,j} for i = 1..m, with the flows leaving it along its
// row, f2_{k,j,l} for l = 1..n, each step taking the smaller remaining
// amount.  That greedy rule is the north-west-corner coupling of the two
// sequences: with P_i, Q_l their running totals, source i and target l
// exchange the overlap of (P_{i-1}, P_i] and (Q_{l-1}, Q_l].  One wave owns
// one bin: it stages both running totals in LDS (FP64).  The entries are the
// segments between consecutive values of the merged totals; the wave takes
// them 64 at a time (merge-path search per lane, a ballot to skip empty
// ones), so both the count and the write pass are balanced across lanes and
// the write is contiguous.  The scaled marginal passes walk each source's
// (or target's) overlaps from a binary-searched start.  Entries are counted,
// offsets come from a scan, and the write pass emits them in a fixed order:
// bins in (k*n + j) order, then source i, then target l.  The flows are the
// clipped max(x_bar, 0) of the solution.
//
// Repair (the algorithm assumes an exactly optimal, feasible flow): rows
// whose total exceeds mu1 are scaled down, then columns above mu2, and the
// remaining row and column deficits are coupled north-west-corner in bin
// order.  All marginals are computed with fixed-order sums (no atomics).
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/hot.h"
#include "hot_internal.h"
#include "hot_runtime.h"

namespace hot {

namespace {

constexpr int kScanBlock = 1024;  // elements per block of the scans

__device__ inline double wave_sum_r(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Clipped flows in unpadded slab layout: F1^(j)[k][i] at j*m*m + k*m + i,
// F2^(k)[j][l] at m*m*n + k*n*n + j*n + l.
template <typename T>
__global__ void k_clip_flows(const PairGeo* __restrict__ geo, const PairCtl* __restrict__ ctl,
                             int pair, const T* __restrict__ sb0, const T* __restrict__ sb1,
                             const T* __restrict__ sb2, const double* __restrict__ ab,
                             double* __restrict__ w) {
  const PairGeo G = geo[pair];
  const PairCtl c = ctl[pair];
  const int m = G.m, n = G.n;
  const int64_t N1 = (int64_t)m * m * n, N = N1 + (int64_t)m * n * n;
  const T* s = c.src == 0 ? sb0 : (c.src == 1 ? sb1 : sb2);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int fam = e < N1 ? 0 : 1;
    const FamGeo F = G.f[fam];
    const int64_t r = fam == 0 ? e : e - N1;
    const int L = F.L;
    const int q = (int)(r % L);
    const int64_t t = r / L;
    const int p = (int)(t % L);
    const int slab = (int)(t / L);
    const double sv = (double)s[F.soff + ((int64_t)slab * L + p) * F.P + q];
    const double* al = ab + F.aboff + (int64_t)slab * 2 * L;
    const double* X = fam_x(ab, F);
    const double d = X[p] - X[q];
    const double g = d * d - al[p] - al[L + q];
    const double x = c.sigma * (sv - g);
    w[e] = x > 0.0 ? x : 0.0;
  }
}

// LDS running totals of one bin: P[0..m] over sources, Q[0..n] over targets.
__device__ inline void stage_prefix(const double* __restrict__ src, int len, double* out,
                                    int lane) {
  for (int t = lane; t < len; t += 64) out[1 + t] = src[t];
  if (lane == 0) out[0] = 0.0;
  __syncthreads();
  const int chunk = (len + 63) / 64;
  const int b0 = min(len, lane * chunk), b1 = min(len, b0 + chunk);
  double loc = 0.0;
  for (int t = b0; t < b1; ++t) loc += out[1 + t];
  double incl = loc;
  for (int off = 1; off < 64; off <<= 1) {
    const double v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  double run = __shfl_up(incl, 1, 64);
  if (lane == 0) run = 0.0;
  __syncthreads();
  for (int t = b0; t < b1; ++t) {
    run += out[1 + t];
    out[1 + t] = run;
  }
  __syncthreads();
  // The lanes' totals are rounded in different orders, so where flows are
  // zero a total can sit a rounding step below its predecessor.  A running
  // maximum (exact in any order) makes the totals nondecreasing, as the
  // searches over them assume.
  double mx = 0.0;
  for (int t = b0; t < b1; ++t) mx = fmax(mx, out[1 + t]);
  for (int off = 1; off < 64; off <<= 1) {
    const double v = __shfl_up(mx, off, 64);
    if (lane >= off) mx = fmax(mx, v);
  }
  double rm = __shfl_up(mx, 1, 64);
  if (lane == 0) rm = 0.0;
  for (int t = b0; t < b1; ++t) {
    rm = fmax(rm, out[1 + t]);
    out[1 + t] = rm;
  }
  __syncthreads();
}

// smallest index l in [0, n) with Q[l+1] > v, or n
__device__ inline int first_above(const double* Q, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (Q[mid + 1] > v) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// smallest index l in [0, n] with l == n or Q[l] >= v (Q nondecreasing)
__device__ inline int count_below(const double* Q, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (Q[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

enum RecPass { PASS_COUNT = 0, PASS_COLSCALED = 1, PASS_BOTHSCALED = 2, PASS_WRITE = 3 };

// The bin's coupling entries in order, 64 candidates per call.  Candidate t
// (t < m + n) is the segment (e_{t-1}, e_t] between consecutive values of the
// merged running totals {P[1..m]} and {Q[1..n]} (e_{-1} = 0); it is an entry
// when it has positive length and lies inside both totals: then it is the
// overlap of source i = #{P[1..m] <= e_{t-1}} and target l likewise, exactly
// min(P[i+1], Q[l+1]) - max(P[i], Q[l]).  Entries come out in the order of
// Algorithm 1's walk (source, then target), and a wave writes them to
// consecutive positions.  `prev` carries e of the previous chunk's last lane.
struct Seg {
  bool ok;
  int i, l;
  double lo, hi;  // the segment (lo, hi]
};
__device__ inline Seg bin_segment(const double* P, const double* Q, int m, int n, int t,
                                  int lane, double& prev) {
  double e = 0.0;
  if (t < m + n) {
    // merge path: a of the k = t + 1 smallest come from P (ties: P first)
    const int k = t + 1;
    int lo = max(0, k - n), hi = min(k, m);
    while (lo < hi) {
      const int a = (lo + hi) >> 1;
      if (P[a + 1] <= Q[k - a]) lo = a + 1; else hi = a;
    }
    e = fmax(P[lo], Q[k - lo]);
  }
  double u = __shfl_up(e, 1, 64);
  if (lane == 0) u = prev;
  prev = __shfl(e, 63, 64);
  Seg sg;
  sg.ok = false;
  sg.i = m;
  sg.l = n;
  sg.lo = u;
  sg.hi = e;
  if (t < m + n && e > u) {
    sg.i = first_above(P, m, u);
    sg.l = first_above(Q, n, u);
    sg.ok = sg.i < m && sg.l < n;
  }
  return sg;
}

// One wave per bin (k, j), item = k*n + j.
template <int PASS>
__global__ __launch_bounds__(64) void k_rec_bin(int m, int n, const double* __restrict__ w,
                                                double* __restrict__ mt,
                                                long long* __restrict__ counts,
                                                const long long* __restrict__ offsets,
                                                const double* __restrict__ rho_r,
                                                const double* __restrict__ rho_c,
                                                int32_t* __restrict__ osrc,
                                                int32_t* __restrict__ odst,
                                                double* __restrict__ omass) {
  extern __shared__ double lds[];
  const int item = blockIdx.x;
  const int k = item / n, j = item % n;
  const int lane = threadIdx.x;
  const int64_t N1 = (int64_t)m * m * n;
  const double* a = w + (int64_t)j * m * m + (int64_t)k * m;       // f1_{., k, j}
  const double* b = w + N1 + (int64_t)k * n * n + (int64_t)j * n;  // f2_{k, j, .}
  double* P = lds;
  double* Q = lds + (m + 1);
  stage_prefix(a, m, P, lane);
  stage_prefix(b, n, Q, lane);
  // scale factors of this bin's sources and targets (small, L2-resident)
  const double* R = PASS != PASS_COUNT ? rho_r + (int64_t)j * m : nullptr;
  const double* C = PASS >= PASS_BOTHSCALED ? rho_c + (int64_t)k * n : nullptr;
  const double PT = P[m], QT = Q[n];
  double* m1 = mt + (int64_t)j * m * m + (int64_t)k * m;
  double* m2 = mt + N1 + (int64_t)k * n * n + (int64_t)j * n;
  if (PASS == PASS_COUNT) {
    // matched amount of source i: its interval clipped to (0, QT]; of target
    // l likewise clipped to (0, PT]
    for (int i = lane; i < m; i += 64) m1[i] = fmax(0.0, fmin(P[i + 1], QT) - fmin(P[i], QT));
    for (int l = lane; l < n; l += 64) m2[l] = fmax(0.0, fmin(Q[l + 1], PT) - fmin(Q[l], PT));
    long long cnt = 0;
    double prev = 0.0;
    for (int t0 = 0; t0 < m + n; t0 += 64) {
      const Seg sg = bin_segment(P, Q, m, n, t0 + lane, lane, prev);
      cnt += __popcll(__ballot(sg.ok));
    }
    if (lane == 0) counts[item] = cnt;
  } else if (PASS == PASS_COLSCALED) {
    // target-centric: sum_i pi_{i,l} rho_r(i,j)
    for (int l = lane; l < n; l += 64) {
      const double lo = Q[l], hi = Q[l + 1];
      double acc = 0.0;
      if (hi > lo) {
        const int i_end = count_below(P, m, hi);  // the overlaps form one run of sources
#pragma unroll 4
        for (int i = first_above(P, m, lo); i < i_end; ++i) {
          const double ov = fmin(P[i + 1], hi) - fmax(P[i], lo);
          if (ov > 0.0) acc += ov * R[i];
        }
      }
      m2[l] = acc;
    }
  } else if (PASS == PASS_BOTHSCALED) {
    for (int i = lane; i < m; i += 64) {
      const double lo = P[i], hi = P[i + 1];
      double acc = 0.0;
      if (hi > lo) {
        const int l_end = count_below(Q, n, hi);  // the overlaps form one run of targets
#pragma unroll 4
        for (int l = first_above(Q, n, lo); l < l_end; ++l) {
          const double ov = fmin(hi, Q[l + 1]) - fmax(lo, Q[l]);
          if (ov > 0.0) acc += ov * R[i] * C[l];
        }
      }
      m1[i] = acc;
    }
    for (int l = lane; l < n; l += 64) {
      const double lo = Q[l], hi = Q[l + 1];
      double acc = 0.0;
      if (hi > lo) {
        const int i_end = count_below(P, m, hi);  // the overlaps form one run of sources
#pragma unroll 4
        for (int i = first_above(P, m, lo); i < i_end; ++i) {
          const double ov = fmin(P[i + 1], hi) - fmax(P[i], lo);
          if (ov > 0.0) acc += ov * R[i] * C[l];
        }
      }
      m2[l] = acc;
    }
  } else {  // PASS_WRITE: the entries in order, 64 candidates per step
    long long base = offsets[item];
    double prev = 0.0;
    for (int t0 = 0; t0 < m + n; t0 += 64) {
      const Seg sg = bin_segment(P, Q, m, n, t0 + lane, lane, prev);
      const unsigned long long mask = __ballot(sg.ok);
      if (sg.ok) {
        const long long pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        osrc[pos] = sg.i * n + j;
        odst[pos] = k * n + sg.l;
        omass[pos] = (sg.hi - sg.lo) * R[sg.i] * C[sg.l];
      }
      base += __popcll(mask);
    }
  }
}

// Column sums of every slab of an unpadded slab-layout buffer:
// out[0 .. n*m): F1 slab j column i at j*m + i; out[n*m ..): F2 slab k column l.
__global__ __launch_bounds__(256) void k_slab_colsum(int m, int n, const double* __restrict__ mt,
                                                     double* __restrict__ out) {
  const int slab = blockIdx.x;  // 0..n-1: F1 slabs; n..n+m-1: F2 slabs
  const int64_t M = (int64_t)m * n, N1 = (int64_t)m * m * n;
  const bool f1 = slab < n;
  const int L = f1 ? m : n;
  const double* base = f1 ? mt + (int64_t)slab * m * m : mt + N1 + (int64_t)(slab - n) * n * n;
  double* o = f1 ? out + (int64_t)slab * m : out + M + (int64_t)(slab - n) * n;
  for (int q = threadIdx.x; q < L; q += 256) {
    double acc = 0.0;
    for (int p = 0; p < L; ++p) acc += base[(int64_t)p * L + q];
    o[q] = acc;
  }
}

// rho = mu / sum where sum > mu, else 1 (out[q] for q in [0, M)); err[q] = |sum - mu|.
__global__ void k_scale_down(const double* __restrict__ sum, const double* __restrict__ mu,
                             int64_t M, double* __restrict__ rho, double* __restrict__ err) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < M;
       q += (int64_t)gridDim.x * blockDim.x) {
    const double s = sum[q], u = mu[q];
    rho[q] = s > u ? u / s : 1.0;
    err[q] = fabs(s - u);
  }
}

// Row deficits in bin order (source bin i*n + j from the [j][i] layout) and
// column deficits ([k][l] is already bin order).
__global__ void k_deficits(int m, int n, const double* __restrict__ r2, const double* __restrict__ c2,
                           const double* __restrict__ mu1T, const double* __restrict__ mu2,
                           double* __restrict__ er, double* __restrict__ ec) {
  const int64_t M = (int64_t)m * n;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < M;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(q / n), j = (int)(q % n);
    const int64_t jt = (int64_t)j * m + i;
    er[q] = fmax(0.0, mu1T[jt] - r2[jt]);
    ec[q] = fmax(0.0, mu2[q] - c2[q]);
  }
}

// North-west-corner coupling of the deficits: er / ec with running totals
// Er / Ec (M+1 entries each).
template <bool WRITE>
__global__ void k_nw(int64_t M, const double* __restrict__ Er, const double* __restrict__ Ec,
                     long long* __restrict__ counts, const long long* __restrict__ offsets,
                     int32_t* __restrict__ osrc, int32_t* __restrict__ odst,
                     double* __restrict__ omass) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < M;
       s += (int64_t)gridDim.x * blockDim.x) {
    const double lo = Er[s], hi = Er[s + 1];
    long long cnt = 0;
    long long pos = WRITE ? offsets[s] : 0;
    if (hi > lo) {
      int64_t a = 0, b = M;  // first t with Ec[t+1] > lo
      while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (Ec[mid + 1] > lo) b = mid; else a = mid + 1;
      }
      for (int64_t t = a; t < M && Ec[t] < hi; ++t) {
        const double ov = fmin(hi, Ec[t + 1]) - fmax(lo, Ec[t]);
        if (ov > 0.0) {
          if (WRITE) {
            osrc[pos] = (int32_t)s;
            odst[pos] = (int32_t)t;
            omass[pos] = ov;
            ++pos;
          } else {
            ++cnt;
          }
        }
      }
    }
    if (!WRITE) counts[s] = cnt;
  }
}

// Final marginal L1 errors: row sums r2 (layout [j][i]) plus the coupled row
// deficit, column sums c2 plus the coupled column deficit.
__global__ void k_final_err(int m, int n, const double* __restrict__ r2,
                            const double* __restrict__ c2, const double* __restrict__ mu1T,
                            const double* __restrict__ mu2, const double* __restrict__ Er,
                            const double* __restrict__ Ec, double* __restrict__ er_out,
                            double* __restrict__ ec_out) {
  const int64_t M = (int64_t)m * n;
  const double T = fmin(Er[M], Ec[M]);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < M;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(q / n), j = (int)(q % n);
    const int64_t jt = (int64_t)j * m + i;
    const double addr = fmax(0.0, fmin(Er[q + 1], T) - fmin(Er[q], T));
    const double addc = fmax(0.0, fmin(Ec[q + 1], T) - fmin(Ec[q], T));
    er_out[q] = fabs(r2[jt] + addr - mu1T[jt]);
    ec_out[q] = fabs(c2[q] + addc - mu2[q]);
  }
}

// ---- fixed-order sums and scans -------------------------------------------
__global__ __launch_bounds__(256) void k_sum_blocks(const double* __restrict__ in, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  for (int t = threadIdx.x; t < kScanBlock; t += 256)
    if (base + t < n) acc += in[base + t];
  acc = wave_sum_r(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_sum_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += part[b];
    *out = acc;
  }
}

// exclusive scan, blocks of kScanBlock elements; out has n+1 entries
template <typename V>
__global__ __launch_bounds__(256) void k_scan_local(const V* __restrict__ in, int64_t n,
                                                    V* __restrict__ out, V* __restrict__ bsum) {
  __shared__ V wt[4];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * 4;
  V v[4];
  V loc = 0;
  for (int u = 0; u < 4; ++u) {
    v[u] = (base + u < n) ? in[base + u] : (V)0;
    loc += v[u];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  V incl = loc;
  for (int off = 1; off < 64; off <<= 1) {
    const V x = __shfl_up(incl, off, 64);
    if (lane >= off) incl += x;
  }
  if (lane == 63) wt[wave] = incl;
  __syncthreads();
  V woff = 0;
  for (int w2 = 0; w2 < wave; ++w2) woff += wt[w2];
  V run = __shfl_up(incl, 1, 64);
  if (lane == 0) run = 0;
  run += woff;
  for (int u = 0; u < 4; ++u) {
    if (base + u < n) out[base + u] = run;
    run += v[u];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = woff + incl;
}

template <typename V>
__global__ void k_scan_top(V* __restrict__ bsum, int nb, V* __restrict__ total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    V run = 0;
    for (int b = 0; b < nb; ++b) {
      const V x = bsum[b];
      bsum[b] = run;
      run += x;
    }
    *total = run;
  }
}

template <typename V>
__global__ void k_scan_add(V* __restrict__ out, int64_t n, const V* __restrict__ bsum) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    out[q] += bsum[q / kScanBlock];
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

template <typename V>
void scan(const V* in, int64_t n, V* out, V* bsum, hipStream_t st) {
  const int nb = (int)((n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_local<V>, dim3(std::max(1, nb)), dim3(256), 0, st, in, n, out, bsum);
  hipLaunchKernelGGL(k_scan_top<V>, dim3(1), dim3(64), 0, st, bsum, std::max(1, nb), out + n);
  hipLaunchKernelGGL(k_scan_add<V>, dim3(grid_for(n)), dim3(256), 0, st, out, n, bsum);
}

void sum_into(const double* in, int64_t n, double* part, double* out, hipStream_t st) {
  const int nb = (int)std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_sum_blocks, dim3(nb), dim3(256), 0, st, in, n, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, st, part, nb, out);
}

// Carves the recovery buffers out of the context's scratch (256-byte
// aligned), growing it when this recovery needs more.  The caller holds
// ctx->rec_mu.
struct ScratchCarver {
  hot_ctx* ctx;
  std::vector<std::pair<void**, size_t>> want;
  template <typename X>
  void add(X** p, size_t count) {
    want.push_back({(void**)p, (std::max<size_t>(count * sizeof(X), 256) + 255) & ~size_t(255)});
  }
  bool commit() {
    size_t need = 0;
    for (const auto& w : want) need += w.second;
    if (need > ctx->rec_bytes) {
      if (ctx->rec_buf) (void)hipFree(ctx->rec_buf);
      ctx->rec_buf = nullptr;
      ctx->rec_bytes = 0;
      if (hipMalloc(&ctx->rec_buf, need) != hipSuccess) {
        (void)hipGetLastError();
        ctx->rec_buf = nullptr;
        return false;
      }
      ctx->rec_bytes = need;
    }
    char* base = (char*)ctx->rec_buf;
    for (const auto& w : want) {
      *w.first = base;
      base += w.second;
    }
    return true;
  }
};

}  // namespace

}  // namespace hot

using namespace hot;

extern "C" hot_status hot_recover_plan(hot_ctx* ctx, const hot_solution* sol, hot_stream_t stream,
                                       int32_t* src, int32_t* dst, double* mass,
                                       int64_t capacity, int64_t* nnz, double* marg_err) {
  if (!ctx || !sol || !src || !dst || !mass || !nnz) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  const int m = sol->m, n = sol->n;
  const int64_t M = (int64_t)m * n;
  const int64_t N1 = (int64_t)m * m * n, N = N1 + (int64_t)m * n * n;
  if (capacity < hot_plan_capacity(m, n)) {
    ctx->err = "plan capacity below hot_plan_capacity(m, n)";
    return HOT_E_INVALID;
  }
  Workspace& ws = *sol->ws;
  const PairGeo& g = ws.lay.geo[sol->pair];
  const double* mu1T = ws.arr + arr_mu1T(g);
  const double* mu2 = ws.arr + arr_mu2(g);
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> rec_lock(ctx->rec_mu);  // the scratch is the context's
  double *w, *mt, *sums, *sums2, *rho_r, *rho_c, *err, *er, *ec, *Er, *Ec, *fb, *part, *res;
  long long *counts, *offs, *ncounts, *noffs, *ibsum;
  const int64_t nbs = (std::max(N, M) + kScanBlock - 1) / kScanBlock + 2;
  ScratchCarver B{ctx, {}};
  B.add(&w, N); B.add(&mt, N); B.add(&sums, 2 * M); B.add(&sums2, 2 * M);
  B.add(&rho_r, M); B.add(&rho_c, M); B.add(&err, M); B.add(&er, M); B.add(&ec, M);
  B.add(&Er, M + 1); B.add(&Ec, M + 1); B.add(&fb, nbs); B.add(&part, nbs); B.add(&res, 8);
  B.add(&counts, M); B.add(&offs, M + 1); B.add(&ncounts, M); B.add(&noffs, M + 1);
  B.add(&ibsum, nbs);
  if (!B.commit()) {
    ctx->err = "recovery workspace allocation failed";
    return HOT_E_NOMEM;
  }
  const LaunchArgs& a = ws.args;
  const int pair = sol->pair;
  if (a.fp32)
    hipLaunchKernelGGL(k_clip_flows<float>, dim3(grid_for(N)), dim3(256), 0, st, a.geo, a.ctl[0],
                       pair, (const float*)a.sb[0], (const float*)a.sb[1], (const float*)a.sb[2],
                       a.ab, w);
  else
    hipLaunchKernelGGL(k_clip_flows<double>, dim3(grid_for(N)), dim3(256), 0, st, a.geo,
                       a.ctl[0], pair, (const double*)a.sb[0], (const double*)a.sb[1],
                       (const double*)a.sb[2], a.ab, w);
  const size_t lds = (size_t)(m + n + 2) * sizeof(double);  // P, Q
  // pass A: counts and matched amounts -> raw marginals r (layout [j][i]), c ([k][l])
  hipLaunchKernelGGL(k_rec_bin<PASS_COUNT>, dim3((unsigned)M), dim3(64), lds, st, m, n, w, mt,
                     counts, (const long long*)nullptr, (const double*)nullptr,
                     (const double*)nullptr, (int32_t*)nullptr, (int32_t*)nullptr,
                     (double*)nullptr);
  hipLaunchKernelGGL(k_slab_colsum, dim3(n + m), dim3(256), 0, st, m, n, mt, sums);
  // raw errors and row scale factors
  hipLaunchKernelGGL(k_scale_down, dim3(grid_for(M)), dim3(256), 0, st, sums, mu1T, M, rho_r, err);
  sum_into(err, M, part, res + 0, st);
  // pass B: column sums after the row scaling
  hipLaunchKernelGGL(k_rec_bin<PASS_COLSCALED>, dim3((unsigned)M), dim3(64), lds, st, m, n, w, mt,
                     counts, (const long long*)nullptr, rho_r, (const double*)nullptr,
                     (int32_t*)nullptr, (int32_t*)nullptr, (double*)nullptr);
  hipLaunchKernelGGL(k_slab_colsum, dim3(n + m), dim3(256), 0, st, m, n, mt, sums2);
  hipLaunchKernelGGL(k_scale_down, dim3(grid_for(M)), dim3(256), 0, st, sums2 + M, mu2, M, rho_c,
                     err);
  // raw column error uses the unscaled column sums
  hipLaunchKernelGGL(k_scale_down, dim3(grid_for(M)), dim3(256), 0, st, sums + M, mu2, M, er, err);
  sum_into(err, M, part, res + 1, st);
  // pass C: row and column sums after both scalings
  hipLaunchKernelGGL(k_rec_bin<PASS_BOTHSCALED>, dim3((unsigned)M), dim3(64), lds, st, m, n, w,
                     mt, counts, (const long long*)nullptr, rho_r, rho_c, (int32_t*)nullptr,
                     (int32_t*)nullptr, (double*)nullptr);
  hipLaunchKernelGGL(k_slab_colsum, dim3(n + m), dim3(256), 0, st, m, n, mt, sums2);
  hipLaunchKernelGGL(k_deficits, dim3(grid_for(M)), dim3(256), 0, st, m, n, sums2, sums2 + M,
                     mu1T, mu2, er, ec);
  scan<double>(er, M, Er, fb, st);
  scan<double>(ec, M, Ec, fb, st);
  // offsets of the bin entries and of the coupling entries
  scan<long long>(counts, M, offs, ibsum, st);
  hipLaunchKernelGGL(k_nw<false>, dim3(grid_for(M)), dim3(256), 0, st, M, Er, Ec, ncounts,
                     (const long long*)nullptr, (int32_t*)nullptr, (int32_t*)nullptr,
                     (double*)nullptr);
  scan<long long>(ncounts, M, noffs, ibsum, st);
  long long tot[2] = {0, 0};
  if (hipMemcpyAsync(&tot[0], offs + M, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&tot[1], noffs + M, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    ctx->err = "recovery count copy failed";
    return HOT_E_DEVICE;
  }
  if (tot[0] + tot[1] > capacity) {
    ctx->err = "plan entries exceed capacity";
    return HOT_E_INVALID;
  }
  hipLaunchKernelGGL(k_rec_bin<PASS_WRITE>, dim3((unsigned)M), dim3(64), lds, st, m, n, w, mt,
                     counts, offs, rho_r, rho_c, src, dst, mass);
  hipLaunchKernelGGL(k_nw<true>, dim3(grid_for(M)), dim3(256), 0, st, M, Er, Ec, ncounts, noffs,
                     src + tot[0], dst + tot[0], mass + tot[0]);
  hipLaunchKernelGGL(k_final_err, dim3(grid_for(M)), dim3(256), 0, st, m, n, sums2, sums2 + M,
                     mu1T, mu2, Er, Ec, er, ec);
  sum_into(er, M, part, res + 2, st);
  sum_into(ec, M, part, res + 3, st);
  double errs[4];
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(errs, res, 4 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    ctx->err = "recovery kernels failed";
    return HOT_E_DEVICE;
  }
  *nnz = tot[0] + tot[1];
  if (marg_err)
    for (int q = 0; q < 4; ++q) marg_err[q] = errs[q];
  return HOT_OK;
}

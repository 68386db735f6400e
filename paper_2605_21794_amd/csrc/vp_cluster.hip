// HIP kernels (gfx950) for the decorated-particle initialisation of arXiv 2605.21794,
// Algorithm 1 ("Decorated Particle Initialization") with the periodic moments of the torus
// subsection: k-means of marker particles in (q, p), then one decorated particle per
// non-empty cluster.
//
// Design:
//  * nearest centre: the centres are binned into a uniform (q, p) grid of about one centre
//    per cell (rebuilt every iteration); each marker searches square rings of cells around
//    its own and stops once the ring bound r * min(cell width, cell height) exceeds its best
//    distance.  The result is the exact nearest centre, ties to the lowest centre index,
//    whatever order the cells list their centres in.
//  * per-cluster sums: the marker indices are sorted by cluster with a stable radix sort
//    (so each cluster's members stay in increasing marker order), and one thread adds its
//    cluster's terms in that order.  The sums are therefore those of a sequential pass over
//    the markers, bit for bit, and the centres, the assignments and the moments are
//    reproducible run to run.
//  * every index that reaches memory is clamped or counted exactly: cell coordinates are
//    clamped into the grid, group positions come from exact integer counts.

#include "vp_internal.h"

#include <mutex>

#include <math.h>

namespace vpk {

namespace {

constexpr double kTwoPi = 6.283185307179586;

struct Grid {
  int gx, gp;
  double sx, sp, pmin;  // cell width in q, height in p, lower edge in p
};

__device__ __forceinline__ int grid_cell(const Grid& g, double q, double p, int* cx, int* cy) {
  double fx = floor(q / g.sx);
  double fy = floor((p - g.pmin) / g.sp);
  int x = !(fx >= 0.0) ? 0 : (fx >= (double)(g.gx - 1) ? g.gx - 1 : (int)fx);
  int y = !(fy >= 0.0) ? 0 : (fy >= (double)(g.gp - 1) ? g.gp - 1 : (int)fy);
  *cx = x;
  *cy = y;
  return y * g.gx + x;
}

// ---------------------------------------------------------------- small helpers
__global__ void k_fill_int(int* p, long long n, int v) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Per-block min / max of p (the markers' velocity range), then one block folds them.
__global__ __launch_bounds__(256) void k_minmax_partial(const double* __restrict__ p, long long m,
                                                        double* __restrict__ part) {
  __shared__ double smin[256], smax[256];
  double lo = INFINITY, hi = -INFINITY;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const double v = p[i];
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smin[0];
    part[2 * blockIdx.x + 1] = smax[0];
  }
}

__global__ __launch_bounds__(256) void k_minmax_final(const double* __restrict__ part, int nb,
                                                      double* __restrict__ out) {
  __shared__ double smin[256], smax[256];
  double lo = INFINITY, hi = -INFINITY;
  for (int i = threadIdx.x; i < nb; i += 256) {
    lo = fmin(lo, part[2 * i]);
    hi = fmax(hi, part[2 * i + 1]);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smin[0];
    out[1] = smax[0];
  }
}

// Exclusive prefix sum of n ints into out[0..n] (out[n] = total), one workgroup walking the
// array in chunks of 1024 with a running carry.
__global__ __launch_bounds__(1024) void k_scan_int(const int* __restrict__ in, int n,
                                                   int* __restrict__ out) {
  __shared__ int buf[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int i = base + (int)threadIdx.x;
    const int v = i < n ? in[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
      const int t = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < n) out[i] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

// Large scans in three passes: the sum of every tile of kScanTile ints, an exclusive scan of
// those sums (one workgroup), then every tile scanned on its own and offset by its sum.
constexpr int kScanTile = 4096;  // 1024 threads x 4

__global__ __launch_bounds__(1024) void k_scan_tile_sums(const int* __restrict__ in, int n,
                                                         int* __restrict__ sums) {
  __shared__ int red[16];
  const long long base = (long long)blockIdx.x * kScanTile + 4LL * threadIdx.x;
  int v = 0;
  for (int u = 0; u < 4; ++u)
    if (base + u < n) v += in[base + u];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < 16; ++w) t += red[w];
    sums[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(1024) void k_scan_tiles(const int* __restrict__ in, int n,
                                                     const int* __restrict__ tile_off,
                                                     int* __restrict__ out) {
  __shared__ int buf[1024];
  const long long base = (long long)blockIdx.x * kScanTile + 4LL * threadIdx.x;
  int x[4], t = 0;
  for (int u = 0; u < 4; ++u) {
    x[u] = base + u < n ? in[base + u] : 0;
    t += x[u];
  }
  buf[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan of the per-thread sums
    const int y = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
    __syncthreads();
    buf[threadIdx.x] += y;
    __syncthreads();
  }
  int run = tile_off[blockIdx.x] + buf[threadIdx.x] - t;
  for (int u = 0; u < 4; ++u) {
    if (base + u < n) out[base + u] = run;
    run += x[u];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tile_off[gridDim.x];
}

// ---------------------------------------------------------------- k-means
__global__ void k_init_centres(const double* __restrict__ q, const double* __restrict__ p,
                               const int* __restrict__ init_idx, int k, double* __restrict__ cq,
                               double* __restrict__ cp) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= k) return;
  const int i = init_idx[a];  // checked against [0, m) on the host
  cq[a] = q[i];
  cp[a] = p[i];
}

__global__ void k_cell_count(const double* __restrict__ cq, const double* __restrict__ cp, int k,
                             Grid g, int* __restrict__ cell_of, int* __restrict__ ccnt) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= k) return;
  int cx, cy;
  const int c = grid_cell(g, cq[a], cp[a], &cx, &cy);
  cell_of[a] = c;
  atomicAdd(ccnt + c, 1);
}

__global__ void k_cell_fill(const int* __restrict__ cell_of, int k, const int* __restrict__ coff,
                            int* __restrict__ ccur, int* __restrict__ clist) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= k) return;
  const int c = cell_of[a];
  clist[coff[c] + atomicAdd(ccur + c, 1)] = a;
}

// Nearest centre of each marker by the ring search (see the file comment).
// Markers are taken in the order perm (sorted by grid cell, so that neighbouring lanes
// search the same cells).
__global__ __launch_bounds__(256) void k_assign(const double* __restrict__ q,
                                                const double* __restrict__ p, long long m,
                                                const int* __restrict__ perm,
                                                const double* __restrict__ cq,
                                                const double* __restrict__ cp, Grid g,
                                                const int* __restrict__ coff,
                                                const int* __restrict__ clist,
                                                int* __restrict__ assign) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  const int i = perm[t];
  const double qi = q[i], pi = p[i];
  int cx, cy;
  grid_cell(g, qi, pi, &cx, &cy);
  const double smin = fmin(g.sx, g.sp);
  const int rmax = g.gx > g.gp ? g.gx : g.gp;
  double best = INFINITY;
  int bi = 0x7fffffff;
  for (int r = 0; r <= rmax; ++r) {
    for (int dy = -r; dy <= r; ++dy) {
      const int y = cy + dy;
      if (y < 0 || y >= g.gp) continue;
      const bool edge = dy == -r || dy == r;
      const int step = edge ? 1 : 2 * r;  // interior rows: only the two ends of the ring
      for (int dx = -r; dx <= r; dx += (step > 0 ? step : 1)) {
        const int x = cx + dx;
        if (x < 0 || x >= g.gx) continue;
        const int c = y * g.gx + x;
        for (int t = coff[c]; t < coff[c + 1]; ++t) {
          const int a = clist[t];
          const double dq = qi - cq[a], dp = pi - cp[a];
          const double d2 = dq * dq + dp * dp;
          if (d2 < best || (d2 == best && a < bi)) {
            best = d2;
            bi = a;
          }
        }
      }
    }
    // every centre not yet seen lies at least r * smin away
    const double bound = (double)r * smin;
    if (bi != 0x7fffffff && best < bound * bound * (1.0 - 1e-9)) break;
  }
  // every centre is binned, so the full square found one, unless every distance was NaN
  // (non-finite or zero-weight input): keep the index in range even then
  assign[i] = bi == 0x7fffffff ? 0 : bi;
}

__global__ void k_marker_cells(const double* __restrict__ q, const double* __restrict__ p,
                               long long m, Grid g, int* __restrict__ cells) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int cx, cy;
  cells[i] = grid_cell(g, q[i], p[i], &cx, &cy);
}

__global__ void k_group_count(const int* __restrict__ assign, long long m, int* __restrict__ cnt) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) atomicAdd(cnt + assign[i], 1);
}

// Stable LSD radix sort of (key, value) pairs by 8-bit digits: per-chunk digit counts, a
// digit-major scan of them, then a stable scatter in which each chunk keeps its elements in
// order.  Chunks of kRadixChunk elements, one 256-thread workgroup each.
__global__ __launch_bounds__(256) void k_radix_hist(const int* __restrict__ keys, long long m,
                                                    int shift, int nb, int* __restrict__ hist) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const long long b0 = (long long)blockIdx.x * kRadixChunk;
  const long long e0 = b0 + kRadixChunk < m ? b0 + kRadixChunk : m;
  for (long long i = b0 + threadIdx.x; i < e0; i += 256)
    atomicAdd(cnt + ((keys[i] >> shift) & 255), 1);
  __syncthreads();
  hist[(long long)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_radix_scatter(const int* __restrict__ kin,
                                                       const int* __restrict__ vin, long long m,
                                                       int shift, int nb,
                                                       const int* __restrict__ hoff,
                                                       int* __restrict__ kout,
                                                       int* __restrict__ vout) {
  __shared__ int run[256];
  __shared__ int dig[256];
  run[threadIdx.x] = hoff[(long long)threadIdx.x * nb + blockIdx.x];
  const long long b0 = (long long)blockIdx.x * kRadixChunk;
  const long long e0 = b0 + kRadixChunk < m ? b0 + kRadixChunk : m;
  for (long long s0 = b0; s0 < e0; s0 += 256) {
    const long long i = s0 + threadIdx.x;
    const bool valid = i < e0;
    const int key = valid ? kin[i] : 0;
    const int d = valid ? ((key >> shift) & 255) : -1;
    __syncthreads();  // run[] settled, dig[] free
    dig[threadIdx.x] = d;
    __syncthreads();
    int rank = 0, total = 0;
    for (int t = 0; t < 256; ++t) {
      const int same = dig[t] == d;
      rank += (t < (int)threadIdx.x) & same;
      total += same;
    }
    if (valid) {
      const int pos = run[d] + rank;
      kout[pos] = key;
      vout[pos] = vin[i];
    }
    __syncthreads();  // every thread has read run[d]
    if (valid && rank + 1 == total) run[d] += total;  // the batch's last element of digit d
  }
}

__global__ void k_iota(int* __restrict__ v, long long m) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) v[i] = (int)i;
}

// New centre of each cluster: weighted mean of its members, summed in marker order; a
// cluster with no members keeps its centre.
__global__ void k_centres(const double* __restrict__ q, const double* __restrict__ p,
                          const double* __restrict__ w, const int* __restrict__ off,
                          const int* __restrict__ order, int k, double* __restrict__ cq,
                          double* __restrict__ cp) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= k) return;
  const int b = off[a], e = off[a + 1];
  if (b == e) return;
  double W = 0.0, SQ = 0.0, SP = 0.0;
  for (int t = b; t < e; ++t) {
    const int i = order[t];
    W += w[i];
    SQ += w[i] * q[i];
    SP += w[i] * p[i];
  }
  cq[a] = SQ / W;
  cp[a] = SP / W;
}

// Mini-batch k-means, the weighted batched form of Sculley's update ("Web-scale k-means
// clustering", 2010): gather the batch's markers (indices clamped into [0, m); the host has
// checked them), then move each centre that received members of this batch to the weighted
// mean of every batch member it has received, its old value standing in for the earlier
// ones: v <- v + W, centre <- (centre v_old + S) / v.  W and S are summed over the members
// in batch order (the grouping sort is stable), so the result is that of a sequential pass.
__global__ void k_gather_batch(const double* __restrict__ q, const double* __restrict__ p,
                               const double* __restrict__ w, long long m,
                               const int* __restrict__ idx, int b, double* __restrict__ bq,
                               double* __restrict__ bp, double* __restrict__ bw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= b) return;
  long long i = idx[t];
  i = i < 0 ? 0 : (i >= m ? m - 1 : i);
  bq[t] = q[i];
  bp[t] = p[i];
  bw[t] = w[i];
}

// Count the batch indices outside [0, m) (host check before any use).
__global__ void k_count_bad(const int* __restrict__ idx, long long n, long long m,
                            int* __restrict__ bad) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && (idx[t] < 0 || (long long)idx[t] >= m)) atomicAdd(bad, 1);
}

__global__ void k_minibatch_update(const double* __restrict__ bq, const double* __restrict__ bp,
                                   const double* __restrict__ bw, const int* __restrict__ off,
                                   const int* __restrict__ order, int k, double* __restrict__ cq,
                                   double* __restrict__ cp, double* __restrict__ v) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= k) return;
  const int b = off[a], e = off[a + 1];
  if (b == e) return;
  double W = 0.0, SQ = 0.0, SP = 0.0;
  for (int t = b; t < e; ++t) {
    const int i = order[t];
    W += bw[i];
    SQ += bw[i] * bq[i];
    SP += bw[i] * bp[i];
  }
  const double vo = v[a], vn = vo + W;
  cq[a] = (cq[a] * vo + SQ) / vn;
  cp[a] = (cp[a] * vo + SP) / vn;
  v[a] = vn;
}

// The decorated particle of each non-empty cluster (Algorithm 1): weight, centre member
// nearest the weighted mean (first in marker order on ties), periodic spatial moment and
// velocity moment, all summed in marker order.  flag[a] = 1 for a non-empty cluster.
__global__ void k_moments(const double* __restrict__ q, const double* __restrict__ p,
                          const double* __restrict__ w, const int* __restrict__ off,
                          const int* __restrict__ order, int k, double L,
                          double* __restrict__ tQ, double* __restrict__ tP,
                          double* __restrict__ tqs, double* __restrict__ tps,
                          double* __restrict__ tpsi, int* __restrict__ flag) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= k) return;
  const int b = off[a], e = off[a + 1];
  if (b == e) {
    flag[a] = 0;
    return;
  }
  double W = 0.0, SQ = 0.0, SP = 0.0;
  for (int t = b; t < e; ++t) {
    const int i = order[t];
    W += w[i];
    SQ += w[i] * q[i];
    SP += w[i] * p[i];
  }
  const double zq = SQ / W, zp = SP / W;
  double best = INFINITY;
  int a0 = order[b];
  for (int t = b; t < e; ++t) {
    const int i = order[t];
    const double dq = q[i] - zq, dp = p[i] - zp;
    const double d2 = dq * dq + dp * dp;
    if (d2 < best) {
      best = d2;
      a0 = i;
    }
  }
  const double Qa = q[a0], Pa = p[a0];
  const double half_len = L / kTwoPi;
  double sps = 0.0, sqs = 0.0;
  for (int t = b; t < e; ++t) {
    const int i = order[t];
    sps += w[i] * (half_len * sin(kTwoPi * (Qa - q[i]) / L));
    sqs += w[i] * (Pa - p[i]);
  }
  tQ[a] = Qa;
  tP[a] = Pa;
  tps[a] = sps;
  tqs[a] = -sqs;
  tpsi[a] = W;
  flag[a] = 1;
}

__global__ void k_compact(const int* __restrict__ flag, const int* __restrict__ pos, int k,
                          const double* __restrict__ tQ, const double* __restrict__ tP,
                          const double* __restrict__ tqs, const double* __restrict__ tps,
                          const double* __restrict__ tpsi, double* __restrict__ Q,
                          double* __restrict__ P, double* __restrict__ qs,
                          double* __restrict__ ps, double* __restrict__ psi) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= k || !flag[a]) return;
  const int j = pos[a];
  Q[j] = tQ[a];
  P[j] = tP[a];
  qs[j] = tqs[a];
  ps[j] = tps[a];
  psi[j] = tpsi[a];
}

__global__ void k_copy_int(const int* __restrict__ in, long long n, int* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

unsigned blocks_for(long long n, int tpb) {
  long long b = (n + tpb - 1) / tpb;
  return (unsigned)(b < 1 ? 1 : b);
}

hipError_t fill_int(int* p, long long n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)b), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Exclusive scan of n ints into out[0..n]; tmp holds 2 * (n / kScanTile + 2) ints.
hipError_t scan_int(const int* in, int n, int* out, int* tmp, hipStream_t s) {
  if (n <= kScanTile) {
    hipLaunchKernelGGL(k_scan_int, dim3(1), dim3(1024), 0, s, in, n, out);
    return hipGetLastError();
  }
  const int nt = (n + kScanTile - 1) / kScanTile;
  int* sums = tmp;
  int* toff = tmp + nt + 1;
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(nt), dim3(1024), 0, s, in, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_int, dim3(1), dim3(1024), 0, s, sums, nt, toff);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(1024), 0, s, in, n, toff, out);
  return hipGetLastError();
}

// Ints of scan scratch for scans of up to n elements.
long long scan_tmp_ints(long long n) { return 2 * (n / kScanTile + 2); }

}  // namespace

ClusterWs cluster_layout(long long m, int k, int batch) {
  ClusterWs w{};
  const long long gmax = cluster_max_cells(k);
  size_t o = 0;
  w.cq = o;      o = a256(o + (size_t)k * sizeof(double));
  w.cp = o;      o = a256(o + (size_t)k * sizeof(double));
  w.assign = o;  o = a256(o + (size_t)m * sizeof(int));
  w.cnt = o;     o = a256(o + (size_t)k * sizeof(int));
  w.off = o;     o = a256(o + (size_t)(k + 1) * sizeof(int));
  w.perm = o;    o = a256(o + (size_t)m * sizeof(int));
  w.keys_a = o;  o = a256(o + (size_t)m * sizeof(int));
  w.vals_a = o;  o = a256(o + (size_t)m * sizeof(int));
  w.keys_b = o;  o = a256(o + (size_t)m * sizeof(int));
  w.vals_b = o;  o = a256(o + (size_t)m * sizeof(int));
  w.hist = o;    o = a256(o + (size_t)256 * radix_blocks(m) * sizeof(int));
  w.hoff = o;    o = a256(o + ((size_t)256 * radix_blocks(m) + 1) * sizeof(int));
  w.cell_of = o; o = a256(o + (size_t)k * sizeof(int));
  w.ccnt = o;    o = a256(o + (size_t)gmax * sizeof(int));
  w.coff = o;    o = a256(o + (size_t)(gmax + 1) * sizeof(int));
  w.ccur = o;    o = a256(o + (size_t)gmax * sizeof(int));
  w.clist = o;   o = a256(o + (size_t)k * sizeof(int));
  w.mm = o;      o = a256(o + (size_t)(2 * kClusterMinMaxBlocks + 2) * sizeof(double));
  w.tQ = o;      o = a256(o + (size_t)k * sizeof(double));
  w.tP = o;      o = a256(o + (size_t)k * sizeof(double));
  w.tqs = o;     o = a256(o + (size_t)k * sizeof(double));
  w.tps = o;     o = a256(o + (size_t)k * sizeof(double));
  w.tpsi = o;    o = a256(o + (size_t)k * sizeof(double));
  w.flag = o;    o = a256(o + (size_t)k * sizeof(int));
  w.pos = o;     o = a256(o + (size_t)(k + 1) * sizeof(int));
  {
    long long nmax = 256 * radix_blocks(m);
    if (nmax < k) nmax = k;
    if (nmax < gmax) nmax = gmax;
    w.scan = o;  o = a256(o + (size_t)scan_tmp_ints(nmax) * sizeof(int));
  }
  // mini-batch regions (batch <= m: the batch's assignment and grouping reuse the marker
  // arrays above)
  const size_t nb = batch > 0 ? (size_t)batch : 0;
  w.v = o;       o = a256(o + (batch > 0 ? (size_t)k : 0) * sizeof(double));
  w.bq = o;      o = a256(o + nb * sizeof(double));
  w.bp = o;      o = a256(o + nb * sizeof(double));
  w.bw = o;      o = a256(o + nb * sizeof(double));
  w.bperm = o;   o = a256(o + nb * sizeof(int));
  w.bad = o;     o = a256(o + sizeof(int));
  w.total = o;
  return w;
}

// ---------------------------------------------------------------- allocation-free workspace
// The workspace of vp_cluster_markers_static.  A file-scope device array: each device the
// library runs on holds its own copy for the life of the process.  In host code the array's
// name is only a stand-in for the symbol, never a device address: its address on a device
// comes from hipGetSymbolAddress, taken once per device with that device current and kept.
static __device__ __align__(256) unsigned char scratch[VP_CLUSTER_STATIC_BYTES];

hipError_t cluster_static_workspace(void** ptr_out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptrs[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptrs[dev] = p;
  }
  *ptr_out = ptrs[dev];
  return hipSuccess;
}

hipError_t cluster_count_bad(const int* idx, long long n, long long m, void* ws,
                             const ClusterWs& w, int* host_bad, hipStream_t s) {
  int* bad = reinterpret_cast<int*>(static_cast<char*>(ws) + w.bad);
  hipError_t e = fill_int(bad, 1, 0, s);
  if (e != hipSuccess) return e;
  if (n > 0) {
    hipLaunchKernelGGL(k_count_bad, dim3(blocks_for(n, 256)), dim3(256), 0, s, idx, n, m, bad);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(host_bad, bad, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return e;
  return hipStreamSynchronize(s);
}

hipError_t cluster_p_range(const double* p, long long m, void* ws, const ClusterWs& w,
                           double* host_minmax, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  double* part = reinterpret_cast<double*>(base + w.mm);
  double* res = part + 2 * kClusterMinMaxBlocks;
  long long nb = (m + 255) / 256;
  if (nb > kClusterMinMaxBlocks) nb = kClusterMinMaxBlocks;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_minmax_partial, dim3((unsigned)nb), dim3(256), 0, s, p, m, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(256), 0, s, part, (int)nb, res);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(host_minmax, res, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// Stable sort of the marker indices 0..m-1 by keys (values below 2^bits) with 8-bit LSD
// passes; keys_a holds the keys on entry (overwritten).  *out = the sorted indices (one of
// vals_a / vals_b).
static hipError_t sort_indices(long long m, int bits, int* keys_a, int* vals_a, int* keys_b,
                               int* vals_b, int* hist, int* hoff, int* stmp, int** out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(blocks_for(m, 256)), dim3(256), 0, s, vals_a, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = (int)((m + kRadixChunk - 1) / kRadixChunk);
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(256), 0, s, keys_a, m, shift, nb, hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_int(hist, 256 * nb, hoff, stmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(256), 0, s, keys_a, vals_a, m, shift, nb,
                       hoff, keys_b, vals_b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int* t = keys_a; keys_a = keys_b; keys_b = t;
    t = vals_a; vals_a = vals_b; vals_b = t;
  }
  *out = vals_a;
  return hipSuccess;
}

static int key_bits(long long nkeys) {
  int bits = 1;
  while (bits < 31 && (1LL << bits) < nkeys) ++bits;
  return bits;
}

// Group the markers by their assignment: counts and segment offsets per cluster, and the
// marker indices sorted by cluster (stable, so in marker order within each cluster).
static hipError_t group_markers(long long m, int k, const int* assign, int* cnt, int* off,
                                int* keys_a, int* vals_a, int* keys_b, int* vals_b, int* hist,
                                int* hoff, int* stmp, int** order_out, hipStream_t s) {
  hipError_t e = fill_int(cnt, k, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_count, dim3(blocks_for(m, 256)), dim3(256), 0, s, assign, m, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_int(cnt, k, off, stmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(m, 256)), dim3(256), 0, s, assign, m, keys_a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return sort_indices(m, key_bits(k), keys_a, vals_a, keys_b, vals_b, hist, hoff, stmp,
                      order_out, s);
}

hipError_t cluster_run(const double* q, const double* p, const double* w, long long m, int k,
                       const int* init_idx, const int* batch_idx, int batch, int nbatch,
                       int iters, double L, double pmin, double pmax, void* ws,
                       const ClusterWs& lay, double* Q, double* P, double* qs, double* ps,
                       double* psi, int* assign_out, double* absorbed_out, int* host_n,
                       hipStream_t s) {
  char* base = static_cast<char*>(ws);
  double* cq = reinterpret_cast<double*>(base + lay.cq);
  double* cp = reinterpret_cast<double*>(base + lay.cp);
  int* assign = reinterpret_cast<int*>(base + lay.assign);
  int* cnt = reinterpret_cast<int*>(base + lay.cnt);
  int* off = reinterpret_cast<int*>(base + lay.off);
  int* keys_a = reinterpret_cast<int*>(base + lay.keys_a);
  int* vals_a = reinterpret_cast<int*>(base + lay.vals_a);
  int* keys_b = reinterpret_cast<int*>(base + lay.keys_b);
  int* vals_b = reinterpret_cast<int*>(base + lay.vals_b);
  int* hist = reinterpret_cast<int*>(base + lay.hist);
  int* hoff = reinterpret_cast<int*>(base + lay.hoff);
  int* stmp = reinterpret_cast<int*>(base + lay.scan);
  int* order = nullptr;
  int* cell_of = reinterpret_cast<int*>(base + lay.cell_of);
  int* ccnt = reinterpret_cast<int*>(base + lay.ccnt);
  int* coff = reinterpret_cast<int*>(base + lay.coff);
  int* ccur = reinterpret_cast<int*>(base + lay.ccur);
  int* clist = reinterpret_cast<int*>(base + lay.clist);
  double* tQ = reinterpret_cast<double*>(base + lay.tQ);
  double* tP = reinterpret_cast<double*>(base + lay.tP);
  double* tqs = reinterpret_cast<double*>(base + lay.tqs);
  double* tps = reinterpret_cast<double*>(base + lay.tps);
  double* tpsi = reinterpret_cast<double*>(base + lay.tpsi);
  int* flag = reinterpret_cast<int*>(base + lay.flag);
  int* pos = reinterpret_cast<int*>(base + lay.pos);

  // grid of about one centre per cell over [0, L) x [pmin, pmax]
  Grid g{};
  const double span = pmax > pmin ? pmax - pmin : 1.0;
  const long long gmax = cluster_max_cells(k);
  double cell = sqrt(L * span / (double)k);
  for (;;) {
    const double gx = ceil(L / cell), gp = ceil(span / cell);
    if (gx * gp <= (double)gmax) {
      g.gx = (int)(gx < 1 ? 1 : gx);
      g.gp = (int)(gp < 1 ? 1 : gp);
      break;
    }
    cell *= 1.25;
  }
  g.sx = L / g.gx;
  g.sp = span / g.gp;
  g.pmin = pmin;
  const int G = g.gx * g.gp;

  hipError_t e = hipSuccess;
  // the markers in grid-cell order (the grid stays fixed): the assignment's visiting order
  int* perm = reinterpret_cast<int*>(base + lay.perm);
  {
    hipLaunchKernelGGL(k_marker_cells, dim3(blocks_for(m, 256)), dim3(256), 0, s, q, p, m, g,
                       keys_a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int* sorted = nullptr;
    if ((e = sort_indices(m, key_bits(G), keys_a, vals_a, keys_b, vals_b, hist, hoff, stmp,
                          &sorted, s)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(m, 256)), dim3(256), 0, s, sorted, m, perm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_init_centres, dim3(blocks_for(k, 256)), dim3(256), 0, s, q, p, init_idx,
                     k, cq, cp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // bin the current centres into the grid (cell lists for the ring search)
  auto bin_centres = [&]() -> hipError_t {
    hipError_t be = fill_int(ccnt, G, 0, s);
    if (be != hipSuccess) return be;
    if ((be = fill_int(ccur, G, 0, s)) != hipSuccess) return be;
    hipLaunchKernelGGL(k_cell_count, dim3(blocks_for(k, 256)), dim3(256), 0, s, cq, cp, k, g,
                       cell_of, ccnt);
    if ((be = hipGetLastError()) != hipSuccess) return be;
    if ((be = scan_int(ccnt, G, coff, stmp, s)) != hipSuccess) return be;
    hipLaunchKernelGGL(k_cell_fill, dim3(blocks_for(k, 256)), dim3(256), 0, s, cell_of, k, coff,
                       ccur, clist);
    return hipGetLastError();
  };
  if (nbatch > 0) {
    // mini-batch updates; the batch's assignment and grouping use the marker arrays (b <= m)
    double* v = reinterpret_cast<double*>(base + lay.v);
    double* bq = reinterpret_cast<double*>(base + lay.bq);
    double* bp = reinterpret_cast<double*>(base + lay.bp);
    double* bw = reinterpret_cast<double*>(base + lay.bw);
    int* bperm = reinterpret_cast<int*>(base + lay.bperm);
    if ((e = launch_fill_zero(v, (size_t)k * sizeof(double), s)) != hipSuccess) return e;
    for (int t = 0; t < nbatch; ++t) {
      if ((e = bin_centres()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_gather_batch, dim3(blocks_for(batch, 256)), dim3(256), 0, s, q, p, w,
                         m, batch_idx + (size_t)t * batch, batch, bq, bp, bw);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      // visit the batch in grid-cell order (a random batch in its own order would send the
      // lanes of a wavefront to unrelated cells); the order does not change any result
      hipLaunchKernelGGL(k_marker_cells, dim3(blocks_for(batch, 256)), dim3(256), 0, s, bq, bp,
                         (long long)batch, g, keys_a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      int* sorted = nullptr;
      if ((e = sort_indices(batch, key_bits(G), keys_a, vals_a, keys_b, vals_b, hist, hoff, stmp,
                            &sorted, s)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(batch, 256)), dim3(256), 0, s, sorted,
                         (long long)batch, bperm);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_assign, dim3(blocks_for(batch, 256)), dim3(256), 0, s, bq, bp,
                         (long long)batch, bperm, cq, cp, g, coff, clist, assign);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = group_markers(batch, k, assign, cnt, off, keys_a, vals_a, keys_b, vals_b, hist,
                             hoff, stmp, &order, s)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(k_minibatch_update, dim3(blocks_for(k, 64)), dim3(64), 0, s, bq, bp, bw,
                         off, order, k, cq, cp, v);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (absorbed_out) {
      if ((e = hipMemcpyAsync(absorbed_out, v, (size_t)k * sizeof(double),
                              hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return e;
    }
  }
  for (int it = 0; it <= iters; ++it) {
    if ((e = bin_centres()) != hipSuccess) return e;
    // assign, group
    hipLaunchKernelGGL(k_assign, dim3(blocks_for(m, 256)), dim3(256), 0, s, q, p, m, perm, cq,
                       cp, g, coff, clist, assign);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = group_markers(m, k, assign, cnt, off, keys_a, vals_a, keys_b, vals_b, hist, hoff,
                           stmp, &order, s)) != hipSuccess)
      return e;
    if (it < iters) {  // move the centres; the last pass only assigns
      hipLaunchKernelGGL(k_centres, dim3(blocks_for(k, 64)), dim3(64), 0, s, q, p, w, off, order,
                         k, cq, cp);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_moments, dim3(blocks_for(k, 64)), dim3(64), 0, s, q, p, w, off, order, k,
                     L, tQ, tP, tqs, tps, tpsi, flag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_int(flag, k, pos, stmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_compact, dim3(blocks_for(k, 256)), dim3(256), 0, s, flag, pos, k, tQ, tP,
                     tqs, tps, tpsi, Q, P, qs, ps, psi);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (assign_out) {
    hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(m, 256)), dim3(256), 0, s, assign, m,
                       assign_out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(host_n, pos + k, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return e;
  return hipStreamSynchronize(s);
}

}  // namespace vpk

// HIP kernels (gfx950) for the decorated-particle cycle of arXiv 2605.21794, Section 5:
// deposit of the monopole + dipole load (eq. rhs-assembly), periodic P1 Poisson solve with
// the zero-mean gauge (eq. lin-sys), gather of E = -phi_h' and of the projected phi_h'',
// and the kick / drift sub-flows of eq. sw-evolution.
//
// Layout: particles are five structure-of-arrays streams; one workgroup owns one tile of
// consecutive particles of one instance, so every load and store is coalesced.  The load
// vector is accumulated into an LDS-private copy of the grid (float64 LDS atomics, or float32
// (hi, lo) two-sum pairs under a 64-bit compare-and-swap, or float32 atomics in the naive
// mode), and each tile adds its grid into one of the instance's spread global accumulator
// copies.  The fused step needs no grid-wide wait: the accumulators form a ring of three
// entries, and every workgroup of the next launch solves the field of the entry the previous
// launch filled (a few microseconds of LDS work that overlap its first particle loads), so
// one kernel per step advances every instance and the kernel boundary is the only barrier.
//
// Rounding: every kernel is compiled without floating-point contraction, and the float64
// particle arithmetic follows the same operation order as the plain CPU definition, so the
// float64 push is bitwise reproducible from the same inputs; only sums differ in order.

#include "vp_internal.h"

#include <math.h>

namespace vpk {

template <int MODE> struct StateType { using T = double; };
template <> struct StateType<kFP32Comp> { using T = float; };
template <> struct StateType<kFP32> { using T = float; };
template <> struct StateType<kFP32TwoSum> { using T = float; };

// Global-memory pointers are spelled in address space 1: pointers read out of the instance
// table would otherwise be generic, and generic (flat) accesses count against the LDS wait
// counter too, so every LDS wait would also drain the in-flight particle traffic.
#define VPG __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ VPG T* gp(void* p) { return (VPG T*)p; }
template <typename T>
__device__ __forceinline__ VPG T* gp(T* p) { return (VPG T*)p; }
// device-scope (all XCDs) atomics and coherent loads / stores
__device__ __forceinline__ void gadd(VPG double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gadd(VPG float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double gld(VPG double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float gld(VPG float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gst(VPG double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gst(VPG float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads of data that other workgroups of the same launch wrote (DEV = true: the persistent
// step) go through device-scope atomic loads, which no stale cache line can answer.
template <bool DEV, typename T>
__device__ __forceinline__ T ldx(VPG T* p) {
  if constexpr (DEV) return gld(p);
  else return *p;
}
template <bool DEV, typename T>
__device__ __forceinline__ void stx(VPG T* p, T v) {
  if constexpr (DEV) gst(p, v);
  else *p = v;
}

// Streaming access to the particle arrays: every element is read and written once per step,
// so the loads and stores are marked non-temporal (they do not displace cached grid data).
template <typename T>
__device__ __forceinline__ T ntld(const VPG T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void ntst(VPG T* p, T v) { __builtin_nontemporal_store(v, p); }

// Element index of x = Q * Ng / L: floor, clamped to [0, Ng-1] (NaN maps to 0), so an LDS
// index is always in range whatever the state holds.
__device__ __forceinline__ int cell_of(double x, int ng) {
  const double f = floor(x);
  if (!(f >= 0.0)) return 0;
  if (f >= (double)(ng - 1)) return ng - 1;
  return (int)f;
}
__device__ __forceinline__ int cell_of_f(float x, int ng) {
  const float f = floorf(x);
  if (!(f >= 0.0f)) return 0;
  if (f >= (float)(ng - 1)) return ng - 1;
  return (int)f;
}
__device__ __forceinline__ double frac01(double x, int i) {
  double s = x - (double)i;
  s = s < 0.0 ? 0.0 : s;
  s = s > 1.0 ? 1.0 : s;
  return s;
}
__device__ __forceinline__ float frac01_f(float x, int i) {
  float s = x - (float)i;
  s = s < 0.0f ? 0.0f : s;
  s = s > 1.0f ? 1.0f : s;
  return s;
}

// phi_h''(Q) of a particle at mesh coordinate x = Q / h in element i, from the curvature
// array g of the instance's projection: the element value, or for the nodal projections
// the P1 interpolant (1 - s) g_i + s g_{i+1}.  `proj` is uniform over a workgroup.
template <typename F>
__device__ __forceinline__ double curv_at(int proj, const F* g, int i, double x, int ng) {
  const double gi = (double)g[i];
  if (proj == VP_PROJ_ELEM) return gi;
  const double s = frac01(x, i);
  return (1.0 - s) * gi + s * (double)g[(i + 1) & (ng - 1)];
}
template <typename F>
__device__ __forceinline__ float curv_at_f(int proj, const F* g, int i, float x, int ng) {
  const float gi = (float)g[i];
  if (proj == VP_PROJ_ELEM) return gi;
  const float s = frac01_f(x, i);
  return (1.0f - s) * gi + s * (float)g[(i + 1) & (ng - 1)];
}

// The field on a particle of an instance with general options (d.general): the mesh field
// and the projection's curvature when the particles feel their own field (else zero), plus
// the prescribed potential's field -V'(Q) and curvature V''(Q); U gets psi* V(Q) - p* V'(Q)
// of the particle (integer-step Q and p*).  Float64, in the plain definition's order.
// P2 elements: fE holds the field at each element's midpoint and fG the element's exact
// phi_h''; the field is linear on the element, E(s) = fE[i] - h fG[i] (s - 1/2).
template <typename F>
__device__ __forceinline__ void general_field(const InstDev& d, const F* fE, const F* fG, int i,
                                              double x, double Q, double psi, double ps,
                                              double& Ei, double& gi, double& U) {
  Ei = d.self_on ? (double)fE[i] : 0.0;
  gi = d.self_on ? curv_at(d.proj, fG, i, x, d.ng) : 0.0;
  if (d.order == 2 && d.self_on) Ei = Ei - d.h * gi * (frac01(x, i) - 0.5);
  U = 0.0;
  if (d.ext_on) {
    const double ph = d.ext_k * Q;
    const double sn = sin(ph), cs = cos(ph);
    Ei = Ei - d.ext_ak * sn;
    gi = gi + d.ext_akk * cs;
    U = psi * (d.ext_a * (1.0 - cs)) - ps * (d.ext_ak * sn);
  }
}

// Deterministic workgroup sum: fixed shuffle tree per wave, then the wave totals in order.
// `red` holds at least TPB/64 doubles.  Every thread of the workgroup must call it.
template <int TPB>
__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < TPB / 64; ++w) r += red[w];
  return r;
}

// ------------------------------------------------------------------ LDS layout
// [0, 2*Ng) doubles: field E then g (float copies for kFP32); [2*Ng, 2*Ng + nacc):
// accumulator (nacc doubles / packed float (hi, lo) pairs / floats; nacc = Ng, or 2 Ng for
// P2).  The solve reuses [0, 4*Ng).
__host__ __device__ constexpr size_t lds_doubles_per_node() { return 4; }

template <int MODE, int TPB>
__device__ void stage(const InstDev& d, double* fld, double* sacc, bool need_field,
                      bool need_acc) {
  const int ng = d.ng;
  if (need_field) {
    if constexpr (MODE == kFP32) {
      float* f = reinterpret_cast<float*>(fld);
      const VPG float* Ef = gp(d.Ef);
      const VPG float* gf = gp(d.gf);
      for (int j = threadIdx.x; j < ng; j += TPB) {
        f[j] = Ef[j];
        f[ng + j] = gf[j];
      }
    } else {
      const VPG double* E = gp(d.E);
      const VPG double* g = gp(d.g);
      for (int j = threadIdx.x; j < ng; j += TPB) {
        fld[j] = E[j];
        fld[ng + j] = g[j];
      }
    }
  }
  if (need_acc)
    for (int j = threadIdx.x; j < d.nacc; j += TPB) sacc[j] = 0.0;
  __syncthreads();
}

// Add the nodal contribution c into the LDS grid.
template <int MODE>
__device__ __forceinline__ void lds_add(double* sacc, int j, double c) {
  if constexpr (MODE == kFP64 || MODE == kFP32Comp) {
    atomicAdd(sacc + j, c);
  } else {
    // float32 (hi, lo) pair packed in one 64-bit word: c = ch + cl exactly (to float64
    // precision); (hi, lo) <- (fl(hi + ch), lo + (e + cl)) with e the exact rounding error of
    // hi + ch (two-sum), committed with a 64-bit compare-and-swap so the pair stays
    // consistent.  A lane retries only when another lane changed the word in between.
    unsigned long long* w = reinterpret_cast<unsigned long long*>(sacc) + j;
    const float ch = (float)c;
    const float cl = (float)(c - (double)ch);
    unsigned long long old = *w;  // first guess; the compare-and-swap validates it
    while (true) {
      const float hi = __uint_as_float((unsigned)(old & 0xffffffffull));
      const float lo = __uint_as_float((unsigned)(old >> 32));
      const float s = hi + ch;
      const float bp = s - hi;
      const float err = (hi - (s - bp)) + (ch - bp);
      const float nlo = lo + (err + cl);
      const unsigned long long nw =
          (unsigned long long)__float_as_uint(s) | ((unsigned long long)__float_as_uint(nlo) << 32);
      const unsigned long long prev = atomicCAS(w, old, nw);
      if (prev == old) break;
      old = prev;
    }
  }
}

// P2 load of one particle at local coordinate s of element j (eq. galerkin with the
// quadratic basis N0 = (1-s)(1-2s), N1 = 4s(1-s), N2 = s(2s-1) of the element's left vertex,
// midpoint and right vertex): node k gets psi* N_k(s) - p* N_k'(s) / h.  Midpoint j is LDS
// entry ng + j.  With DIP false p* is zero and its terms are left out.
template <int MODE, bool DIP>
__device__ __forceinline__ void deposit_p2(double* sacc, int ng, int j, double s, double psi,
                                           double ps, double inv_h) {
  const double n0 = (1.0 - s) * (1.0 - 2.0 * s), n1 = 4.0 * s * (1.0 - s), n2 = s * (2.0 * s - 1.0);
  if constexpr (DIP) {
    lds_add<MODE>(sacc, j, psi * n0 - ps * ((4.0 * s - 3.0) * inv_h));
    lds_add<MODE>(sacc, ng + j, psi * n1 - ps * ((4.0 - 8.0 * s) * inv_h));
    lds_add<MODE>(sacc, (j + 1) & (ng - 1), psi * n2 - ps * ((4.0 * s - 1.0) * inv_h));
  } else {
    lds_add<MODE>(sacc, j, psi * n0);
    lds_add<MODE>(sacc, ng + j, psi * n1);
    lds_add<MODE>(sacc, (j + 1) & (ng - 1), psi * n2);
  }
}

// Add the LDS grid into accumulator copy `copy` of ring entry r of the instance (device-scope
// atomics; only non-zero nodes).
template <int MODE, int TPB>
__device__ void flush(const InstDev& d, const double* sacc, int r, int copy) {
  const int ng = d.nacc;
  const size_t off = ((size_t)r * VP_MAX_ACC_COPIES + (size_t)copy) * (size_t)ng;
  if constexpr (MODE == kFP32) {
    const float* a = reinterpret_cast<const float*>(sacc);
    VPG float* gacc = gp<float>(d.acc) + off;
    for (int j = threadIdx.x; j < ng; j += TPB) {
      const float v = a[j];
      if (v != 0.0f) gadd(gacc + j, v);
    }
  } else if constexpr (MODE == kFP32TwoSum) {
    const unsigned long long* wv = reinterpret_cast<const unsigned long long*>(sacc);
    VPG double* gacc = gp(d.acc) + off;
    for (int j = threadIdx.x; j < ng; j += TPB) {
      const unsigned long long w = wv[j];
      const double v = (double)__uint_as_float((unsigned)(w & 0xffffffffull)) +
                       (double)__uint_as_float((unsigned)(w >> 32));
      if (v != 0.0) gadd(gacc + j, v);
    }
  } else {
    VPG double* gacc = gp(d.acc) + off;
    for (int j = threadIdx.x; j < ng; j += TPB) {
      const double v = sacc[j];
      if (v != 0.0) gadd(gacc + j, v);
    }
  }
}

// Wavefront collectives built from DPP row moves (VALU, no LDS round trip): a 64-lane
// inclusive scan is row_shr 1, 2, 4, 8 inside each 16-lane row, then row_bcast 15 and 31
// carry the row totals upward.  Out-of-row sources read as zero.  Every lane must be
// active.  The order of additions is fixed, so results do not depend on timing.
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, BOUND_ZERO);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, BOUND_ZERO);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_incl_scan(double x) {
  x += dpp_move<0x111, 0xf, true>(x);   // row_shr:1
  x += dpp_move<0x112, 0xf, true>(x);   // row_shr:2
  x += dpp_move<0x114, 0xf, true>(x);   // row_shr:4
  x += dpp_move<0x118, 0xf, true>(x);   // row_shr:8
  x += dpp_move<0x142, 0xa, false>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_move<0x143, 0xc, false>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ __forceinline__ double wave_bcast63(double x) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), 63);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes; every lane gets the same total.
__device__ __forceinline__ double wave_sum(double v) { return wave_bcast63(wave_incl_scan(v)); }

// Exclusive prefix over lanes of one value per lane.
__device__ __forceinline__ double wave_excl_scan(double v, int /*lane*/) {
  return wave_incl_scan(v) - v;
}

// Radix-2 FFT by one wavefront on (re, im) in LDS, input in bit-reversed order; tw holds
// cos/sin(2 pi k / Ng) for k < Ng/2 (LDS).
__device__ void fft_wave(double* re, double* im, int ng, int m, const double* tw, bool inverse,
                         int lane) {
  for (int s = 1; s <= m; ++s) {
    const int half = 1 << (s - 1);
    const int tstride = ng >> s;
    for (int b = lane; b < (ng >> 1); b += 64) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> (s - 1)) << s) + pos;
      const int i1 = i0 + half;
      const int k = pos * tstride;
      const double c = tw[2 * k];
      const double sn = inverse ? -tw[2 * k + 1] : tw[2 * k + 1];
      const double xr = re[i1], xi = im[i1];
      const double tr = c * xr + sn * xi;  // (c - i sn) (xr + i xi)
      const double ti = c * xi - sn * xr;
      const double ur = re[i0], ui = im[i0];
      re[i0] = ur + tr;
      im[i0] = ui + ti;
      re[i1] = ur - tr;
      im[i1] = ui - ti;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

__device__ void bit_reverse_wave(double* re, double* im, int ng, int m, int lane) {
  for (int j = lane; j < ng; j += 64) {
    const int r = (int)(__brev((unsigned)j) >> (32 - m));
    if (j < r) {
      double t = re[j];
      re[j] = re[r];
      re[r] = t;
      t = im[j];
      im[j] = im[r];
      im[r] = t;
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------ Poisson solve
// Every solve (the prologue of each fused workgroup and the materialising kernel) runs on
// the first kSolveThreads threads with the same node split, so the arithmetic, and hence the
// field, is bitwise the same whatever the workgroup size: thread t owns the contiguous nodes
// [t*per, (t+1)*per), per = max(1, Ng / kSolveThreads).  Sums go through fixed DPP wave
// trees and the four wave totals in order.
constexpr int kSolveThreads = 256;
constexpr int kSolveWaves = kSolveThreads / 64;
constexpr int kSolvePer = VP_MAX_NG / kSolveThreads;
// LDS doubles for the solve's wave totals: mean | scan carries | gauge sums | W | Re E1 |
// Im E1 | K | momentum | charge | U
constexpr int kSolveRed = 10 * kSolveWaves;

__device__ __forceinline__ int ring_next(int r) { return r == kRing - 1 ? 0 : r + 1; }
__device__ __forceinline__ int ring_prev(int r) { return r == 0 ? kRing - 1 : r - 1; }

// Element offset of accumulator copy c of ring entry r (in doubles, or in floats for kFP32).
__device__ __forceinline__ size_t acc_off(const InstDev& d, int r, int c) {
  return ((size_t)r * VP_MAX_ACC_COPIES + (size_t)c) * (size_t)d.nacc;
}

__device__ __forceinline__ int solve_per(int ng) {
  return ng >= kSolveThreads ? ng / kSolveThreads : 1;
}

// What a solving thread loads up front: its nodes' load-vector values and, when the field
// summary is wanted, the Fourier weights cos / sin(2 pi e / Ng) of those nodes.
struct SolveIn {
  double b[kSolvePer];
  double bm[kSolvePer];    // P2: the loads of the midpoints of the same elements
  double c[kSolvePer];
  double s[kSolvePer];
  double kin[kKinFields];  // this thread's share of the previous pass's per-tile sums
};

// Sum over tiles t = tid, tid + kSolveThreads, ... (in that order) of the per-tile kinetic
// sums of ring entry r, four tiles' loads in flight at a time.
// NF = 3 leaves out the prescribed-potential sums (launches without general options).
template <bool DEV, int NF = kKinFields>
__device__ __forceinline__ void load_kin(const InstDev& d, int r, double (&kin)[kKinFields]) {
  kin[0] = kin[1] = kin[2] = kin[3] = 0.0;
  VPG double* base = gp(d.kin) + (size_t)r * d.kin_cap * kKinFields;
  for (int t0 = threadIdx.x; t0 < d.ntiles; t0 += 4 * kSolveThreads) {
    double v[4][kKinFields];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * kSolveThreads;
#pragma unroll
      for (int f = 0; f < kKinFields; ++f) v[u][f] = 0.0;
      if (t < d.ntiles) {
#pragma unroll
        for (int f = 0; f < NF; ++f) v[u][f] = ldx<DEV>(base + (size_t)t * kKinFields + f);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int f = 0; f < NF; ++f) kin[f] += v[u][f];
  }
}

// Copies are loaded in batches of at most eight values in flight per thread (bounded
// registers), and added in copy order.
template <int MODE, int COPIES, int PER, bool DEV>
__device__ __forceinline__ void load_copies(const InstDev& d, int r, int j0,
                                            double (&b)[kSolvePer]) {
  // j0 counts from the start of a copy: nodes [ng, 2 ng) are a P2 instance's midpoints
  constexpr int kBatch = (8 / PER) < COPIES ? (8 / PER) : COPIES;
#pragma unroll
  for (int k = 0; k < PER; ++k) b[k] = 0.0;
#pragma unroll
  for (int c0 = 0; c0 < COPIES; c0 += kBatch) {
    double t[kBatch][PER];
#pragma unroll
    for (int c = 0; c < kBatch; ++c)
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        if constexpr (MODE == kFP32)
          t[c][k] = (double)ldx<DEV>(gp<float>(d.acc) + acc_off(d, r, c0 + c) + j0 + k);
        else
          t[c][k] = ldx<DEV>(gp(d.acc) + acc_off(d, r, c0 + c) + j0 + k);
      }
#pragma unroll
    for (int k = 0; k < PER; ++k)
#pragma unroll
      for (int c = 0; c < kBatch; ++c) b[k] += t[c][k];  // copy order
  }
}

// The node count per thread and the copy count are template parameters, so every load is
// unconditional and all of them are in flight before the first use.
template <int MODE, int PER, bool DEV>
__device__ __forceinline__ void load_node_copies(const InstDev& d, int r, int j0,
                                                 double (&b)[kSolvePer]) {
  switch (d.acc_copies) {
    case 1: load_copies<MODE, 1, PER, DEV>(d, r, j0, b); break;
    case 2: load_copies<MODE, 2, PER, DEV>(d, r, j0, b); break;
    case 3: load_copies<MODE, 3, PER, DEV>(d, r, j0, b); break;
    case 4: load_copies<MODE, 4, PER, DEV>(d, r, j0, b); break;
    default: load_copies<MODE, VP_MAX_ACC_COPIES, PER, DEV>(d, r, j0, b); break;
  }
}

template <int MODE, int PER, bool DEV, bool P2>
__device__ __forceinline__ void solve_load_per(const InstDev& d, int r, int j0, bool want_sum,
                                               SolveIn& in) {
  load_node_copies<MODE, PER, DEV>(d, r, j0, in.b);
  if constexpr (P2)
    if (d.order == 2) load_node_copies<MODE, PER, DEV>(d, r, d.ng + j0, in.bm);
  if (want_sum) {
    const VPG double* tw = gp(d.tw);
    const int halfn = d.ng >> 1;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = j0 + k, t = e & (halfn - 1);
      const double sg = (e < halfn) ? 1.0 : -1.0;  // cos / sin of theta + pi
      in.c[k] = sg * tw[2 * t];
      in.s[k] = sg * tw[2 * t + 1];
    }
  }
}

// Issue the solve's loads (load vector of ring entry r; with want_sum also the Fourier
// weights and the kinetic sums of the previous pass, ring entry r-1): all of them before
// any use, so they overlap other work of the caller.
// P2 = false: no instance of the launch has P2 elements (its midpoint loads are not read).
template <int MODE, bool DEV = false, bool GEN = true, bool P2 = GEN>
__device__ __forceinline__ void solve_load(const InstDev& d, int r, bool want_sum, SolveIn& in) {
  const int ng = d.ng, tid = threadIdx.x;
  const int per = solve_per(ng), j0 = tid * per;
#pragma unroll
  for (int k = 0; k < kSolvePer; ++k) in.b[k] = in.bm[k] = in.c[k] = in.s[k] = 0.0;
  in.kin[0] = in.kin[1] = in.kin[2] = in.kin[3] = 0.0;
  if (tid >= kSolveThreads) return;
  if (j0 < ng) {
    if (per == 1) solve_load_per<MODE, 1, DEV, P2>(d, r, j0, want_sum, in);
    else if (per == 2) solve_load_per<MODE, 2, DEV, P2>(d, r, j0, want_sum, in);
    else solve_load_per<MODE, kSolvePer, DEV, P2>(d, r, j0, want_sum, in);
  }
  if (want_sum) load_kin<DEV, GEN ? kKinFields : 3>(d, ring_prev(r), in.kin);  // waits overlap
}

// Sum of one value per solving thread (fixed DPP tree, then the wave totals in order),
// published through red[slot*kSolveWaves ..] at the caller's next barrier.
__device__ __forceinline__ void solve_wave_total(double v, double* red, int slot) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[slot * kSolveWaves + (threadIdx.x >> 6)] = v;
}
__device__ __forceinline__ double solve_total(const double* red, int slot) {
  return red[slot * kSolveWaves] + red[slot * kSolveWaves + 1] + red[slot * kSolveWaves + 2] +
         red[slot * kSolveWaves + 3];
}

// From the loaded values, compute into LDS:
//   bt_j = b~_j = b_j - mean(b)                          (float64, eq. neutrality);
//   E_e  from A Phi = b~, 1^T Phi = 0: E_e - E_{e-1} = b~_e (row j of A Phi = b~ written with
//        E_e = (Phi_e - Phi_{e+1}) / h) and sum_e E_e = 0, so E_e = S_e + C with
//        S_e = sum_{j=1..e} b~_j and C = -(1/Ng) sum_{j>=1} (Ng - j) b~_j;  or by FFT;
//   g_e  = -(b~_e + b~_{e+1}) / (2h): the lumped L2 projection of E onto P1, differentiated;
//   phi  (only when `phi` is given): nodal potential, zero mean;
// and, with want_sum, sum[0..2] = W = (1/2) h sum_e E_e^2 and
// E1 = (1/Ng) sum_e E_e exp(-2 pi i e / Ng), sum[3..6] = K, momentum, charge, U of the
// previous pass (its per-tile sums in tile order), in every thread.
// `fft` is LDS scratch of 3 Ng doubles (FFT solver only).  All threads of the workgroup call
// it (it holds workgroup barriers; want_sum must be uniform); on return bt, E, g (and phi)
// are visible to all threads.
// P2 elements (GEN only): the background n0 = sum(b) / L is subtracted against each basis
// function's integral, n0 h / 3 = mean / 3 at a vertex and 2 mean / 3 at a midpoint (mean =
// sum(b) / Ng).  Static condensation of the midpoint unknowns, whose rows read
// (1/3h)(16 Phi_m - 8 Phi_e - 8 Phi_{e+1}) = b~_m, turns the vertex rows into the P1 system
// with the load c_e = b~_e + (b~_{m,e-1} + b~_{m,e}) / 2 = b_e + (b_{m,e-1} + b_{m,e}) / 2 -
// mean, solved as above (bt holds c~): E_e is then the field at element e's midpoint and
// g_e = -3 b~_{m,e} / (2h) the exact phi_h'' on the element.  The field is linear on the
// element with slope 3 b~_{m,e} / (2h), so W gains (1/2) h (3/16) sum_e b~_{m,e}^2.  With
// `p2b` given, b~ of the vertices and midpoints go to p2b[0, Ng) and p2b[Ng, 2 Ng).  g holds
// the raw midpoint loads until the final pass.
template <int TPB, bool GEN = true, bool P2 = GEN>
__device__ void solve_compute(const InstDev& d, const SolveIn& in, bool want_sum, double* bt,
                              double* E, double* g, double* red, double* fft, double* phi,
                              double* sum, double* p2b = nullptr) {
  const int ng = d.ng, mask = ng - 1, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int per = solve_per(ng), j0 = tid * per;
  const bool solver_thread = tid < kSolveThreads;           // whole waves
  const bool act = solver_thread && j0 < ng;
  const bool use_fft = d.solver == VP_SOLVE_FFT;
  const bool p2 = P2 && d.order == 2;

  double part = 0.0;
#pragma unroll
  for (int k = 0; k < kSolvePer; ++k)
    if (act && k < per) {
      part += in.b[k];
      if (p2) {
        part += in.bm[k];
        g[j0 + k] = in.bm[k];
      }
    }
  if (solver_thread) {
    solve_wave_total(part, red, 0);
    if (want_sum) {
      solve_wave_total(in.kin[0], red, 6);
      solve_wave_total(in.kin[1], red, 7);
      solve_wave_total(in.kin[2], red, 8);
      if constexpr (GEN) solve_wave_total(in.kin[3], red, 9);
    }
  }
  if (use_fft) {  // twiddles for the wavefront FFT
    const VPG double* tw_g = gp(d.tw);
    for (int j = tid; j < ng; j += TPB) fft[2 * ng + j] = tw_g[j];
  }
  __syncthreads();
  const double mean = solve_total(red, 0) / (double)ng;

  double S[kSolvePer];
  double tot = 0.0, wsum = 0.0, wmid = 0.0;
#pragma unroll
  for (int k = 0; k < kSolvePer; ++k) {
    S[k] = 0.0;
    if (act && k < per) {
      const int j = j0 + k;
      double x;
      if (p2) {
        x = (in.b[k] + 0.5 * (g[(j - 1) & mask] + g[j])) - mean;
        const double bmt = in.bm[k] - (2.0 / 3.0) * mean;
        wmid += bmt * bmt;
        if (p2b) {
          p2b[j] = in.b[k] - mean / 3.0;
          p2b[ng + j] = bmt;
        }
      } else {
        x = in.b[k] - mean;
      }
      bt[j] = x;
      if (j > 0) {
        tot += x;
        wsum += (double)(ng - j) * x;
      }
      S[k] = tot;
    }
  }
  double wp = 0.0, er = 0.0, ei = 0.0;  // field-summary partials of this thread's nodes
  if (!use_fft) {
    double off = 0.0;
    if (solver_thread) {
      const double incl = wave_incl_scan(tot);
      off = incl - tot;
      if (lane == 63) red[kSolveWaves + wid] = incl;
      solve_wave_total(wsum, red, 2);
    }
    __syncthreads();
    if (act) {
      for (int w = 0; w < wid; ++w) off += red[kSolveWaves + w];
      const double C = -solve_total(red, 2) / (double)ng;
#pragma unroll
      for (int k = 0; k < kSolvePer; ++k)
        if (k < per) {
          const double Ee = (S[k] + off) + C;
          E[j0 + k] = Ee;
          wp += Ee * Ee;
          er += Ee * in.c[k];
          ei -= Ee * in.s[k];
        }
    }
    if (want_sum && solver_thread) {
      if (p2) wp += 0.1875 * wmid;
      solve_wave_total(wp, red, 3);
      solve_wave_total(er, red, 4);
      solve_wave_total(ei, red, 5);
    }
  } else {
    __syncthreads();  // b~ and the twiddles in LDS
    if (tid < 64) {
      double* re = fft;
      double* im = fft + ng;
      const double* tw = fft + 2 * ng;
      const int m = d.log2ng;
      for (int j = lane; j < ng; j += 64) {
        re[j] = bt[j];
        im[j] = 0.0;
      }
      __builtin_amdgcn_wave_barrier();
      bit_reverse_wave(re, im, ng, m, lane);
      fft_wave(re, im, ng, m, tw, false, lane);
      const VPG double* il_g = gp(d.inv_lam);
      for (int k = lane; k < ng; k += 64) {
        const double il = il_g[k];
        re[k] = re[k] * il;
        im[k] = im[k] * il;
      }
      __builtin_amdgcn_wave_barrier();
      bit_reverse_wave(re, im, ng, m, lane);
      fft_wave(re, im, ng, m, tw, true, lane);
      const double inv_ng = 1.0 / (double)ng;
      for (int j = lane; j < ng; j += 64) re[j] = re[j] * inv_ng;  // Phi
      __builtin_amdgcn_wave_barrier();
      const double inv_h = d.inv_h;
      for (int e = lane; e < ng; e += 64) {
        E[e] = -(re[(e + 1) & mask] - re[e]) * inv_h;
        if (phi) phi[e] = re[e];
      }
    }
    if (want_sum) {
      __syncthreads();  // E complete
      if (act)
#pragma unroll
        for (int k = 0; k < kSolvePer; ++k)
          if (k < per) {
            const double Ee = E[j0 + k];
            wp += Ee * Ee;
            er += Ee * in.c[k];
            ei -= Ee * in.s[k];
          }
      if (solver_thread) {
        if (p2) wp += 0.1875 * wmid;
        solve_wave_total(wp, red, 3);
        solve_wave_total(er, red, 4);
        solve_wave_total(ei, red, 5);
      }
    }
  }
  __syncthreads();  // bt, E and the summary totals complete
  if (want_sum) {
    sum[0] = 0.5 * d.h * solve_total(red, 3);
    sum[1] = solve_total(red, 4) / (double)ng;
    sum[2] = solve_total(red, 5) / (double)ng;
    sum[3] = solve_total(red, 6);
    sum[4] = solve_total(red, 7);
    sum[5] = solve_total(red, 8);
    sum[6] = GEN ? solve_total(red, 9) : 0.0;
  }
  if (p2) {
    // each thread rewrites only entries it reads (the neighbours' reads ended at a barrier)
    const double bg = (2.0 / 3.0) * mean, a = 1.5 * d.inv_h;
    for (int e = tid; e < ng; e += TPB) g[e] = -(g[e] - bg) * a;
  } else if (d.proj == VP_PROJ_ELEM) {
    const double half_inv_h = 0.5 * d.inv_h;
    for (int e = tid; e < ng; e += TPB) g[e] = -(bt[e] + bt[(e + 1) & mask]) * half_inv_h;
  } else if (d.proj == VP_PROJ_NODAL) {
    const double inv_h = d.inv_h;
    for (int e = tid; e < ng; e += TPB) g[e] = -bt[e] * inv_h;
  } else {
    // g = -M^-1 b~ as a circular convolution with the decaying taps of -M^-1 (uniform
    // loads of the tap table), summed in tap order
    const VPG double* __restrict__ cw = gp(d.cw);
    const int taps = cons_taps(ng), off = cons_off(ng);
    for (int e = tid; e < ng; e += TPB) {
      double a = 0.0;
      for (int t = 0; t < taps; ++t) a += cw[t] * bt[(e - t - off) & mask];
      g[e] = a;
    }
  }
  if (phi && !use_fft) {
    // Phi_e = -h (P_e - mean(P)), P_e = sum_{k<e} E_k; sum_e P_e = sum_k (Ng-1-k) E_k
    double P[kSolvePer];
    double ptot = 0.0, pw = 0.0;
#pragma unroll
    for (int k = 0; k < kSolvePer; ++k) {
      P[k] = 0.0;
      if (act && k < per) {
        const int j = j0 + k;
        P[k] = ptot;
        const double Ej = E[j];
        ptot += Ej;
        pw += (double)(ng - 1 - j) * Ej;
      }
    }
    double poff = 0.0;
    if (solver_thread) {
      const double incl = wave_incl_scan(ptot);
      poff = incl - ptot;
      if (lane == 63) red[kSolveWaves + wid] = incl;
      solve_wave_total(pw, red, 2);
    }
    __syncthreads();
    if (act) {
      for (int w = 0; w < wid; ++w) poff += red[kSolveWaves + w];
      const double Pm = solve_total(red, 2) / (double)ng;
#pragma unroll
      for (int k = 0; k < kSolvePer; ++k)
        if (k < per) phi[j0 + k] = -d.h * ((P[k] + poff) - Pm);
    }
  }
  __syncthreads();
}

// Record of integer step `step` (kinetic and potential sums of that step's pass, field
// summary of its field) into the history ring; flags non-finite values.  One thread.
__device__ void write_record(const InstDev& d, long long step, double K, double mom, double chg,
                             double U, double W, double e1r, double e1i) {
  if (!d.self_on) W = e1r = e1i = 0.0;  // no field of their own acts on the particles
  VPG double* r = gp(d.hist) + (size_t)(step % d.hist_cap) * kHistFields;
  r[0] = (double)step;
  r[1] = (double)step * d.dt;
  r[2] = K;
  r[3] = W;
  r[4] = K + U + W;
  r[5] = chg;
  r[6] = mom;
  r[7] = sqrt(2.0 * W / d.L);
  r[8] = e1r;
  r[9] = e1i;
  r[10] = U;
  if (!isfinite(K) || !isfinite(W) || !isfinite(U)) gp(d.scal)->nonfinite = 1;
}

// ------------------------------------------------------------------ particle passes
// Loop shape shared by the particle kernels: thread t of the workgroup handles particles
// tile.begin + k * TPB + t for k < ppt, four at a time with all loads issued first.
#define VP_TILE_LOOP_BEGIN                                                        \
  for (int k0 = 0; k0 < ppt; k0 += 4) {                                           \
    bool v[4];                                                                    \
    long long idx[4];                                                             \
    _Pragma("unroll") for (int u = 0; u < 4; ++u) {                              \
      const int loc = (k0 + u) * TPB + (int)threadIdx.x;                          \
      v[u] = (k0 + u < ppt) && (loc < tl.count);                                  \
      idx[u] = tl.begin + loc;                                                    \
    }

#define VP_TILE_LOOP_END }

// One particle through one step (eq. sw-evolution as a kick-drift-kick splitting): the
// half-kick still owed from the previous step (pend), the kinetic terms at the integer step,
// this step's half-kick, the drift, and the deposit of the drifted particle into the LDS
// grid (eq. rhs-assembly).  (Q, P, q*, p*) are updated in place in storage precision.  The
// float64 modes compute in float64 from the stored values in the oracle's operation order.
// DIP = false: a monopole-only particle (p* = q* = 0, plain P1 particle-in-cell): the dipole
// terms are left out, which gives the same values as carrying zeros through them.
template <int MODE, typename T, bool DIP = true, bool GEN = true, bool P2 = GEN>
__device__ __forceinline__ void push_particle(const InstDev& d, const double* fE, const double* fG,
                                              double* sacc, int pend, T& Qr, T& Pr, T& qsr,
                                              T& psr, const T psir, double& Ks, double& Ms,
                                              double& Cs, double& Us) {
  const int ng = d.ng;
  if constexpr (MODE == kFP32) {
    float* fa = reinterpret_cast<float*>(sacc);
    const float Lf = (float)d.L, ihf = (float)d.inv_h, dtf = (float)d.dt, hf = 0.5f * dtf;
    float Q = Qr, P = Pr, qs = qsr, ps = psr;
    const float psi = psir;
    const float xq = Q * ihf;
    const int i = cell_of_f(xq, ng);
    float Ei, gi;
    if (!GEN || !d.general) {
      Ei = (float)fE[i];
      gi = DIP ? (float)fG[i] : 0.0f;
    } else {
      double e, g, u;
      general_field(d, fE, fG, i, (double)Q * d.inv_h, (double)Q, (double)psi, (double)ps, e, g,
                    u);
      Ei = (float)e;
      gi = (float)g;
      Us += u;
    }
    if constexpr (DIP) {
      if (pend) { P = P + hf * Ei; qs = qs + hf * ps * gi; }
      const double Pd = P, qd = qs, wd = psi;
      Ks += 0.5 * wd * Pd * Pd + qd * Pd;
      Ms += wd * Pd + qd;
      Cs += wd;
      P = P + hf * Ei;
      qs = qs + hf * ps * gi;
    } else {
      if (pend) P = P + hf * Ei;
      const double Pd = P, wd = psi;
      Ks += 0.5 * wd * Pd * Pd;
      Ms += wd * Pd;
      Cs += wd;
      P = P + hf * Ei;
    }
    float Qn = Q + dtf * P;
    if (Qn < 0.0f) Qn += Lf;
    if (Qn >= Lf) Qn -= Lf;
    if constexpr (DIP) ps = ps - dtf * qs;
    const float x = Qn * ihf;
    const int j = cell_of_f(x, ng);
    const float s = frac01_f(x, j);
    if constexpr (DIP) {
      atomicAdd(fa + j, psi * (1.0f - s) + ps * ihf);
      atomicAdd(fa + ((j + 1) & (ng - 1)), psi * s - ps * ihf);
    } else {
      atomicAdd(fa + j, psi * (1.0f - s));
      atomicAdd(fa + ((j + 1) & (ng - 1)), psi * s);
    }
    Qr = Qn; Pr = P;
    if constexpr (DIP) { qsr = qs; psr = ps; }
  } else {
    const double L = d.L, inv_h = d.inv_h, dt = d.dt, half = 0.5 * d.dt;
    const double Q = Qr, psi = psir;
    double P = Pr, qs = qsr, ps = psr;
    const double xq = Q * inv_h;
    const int i = cell_of(xq, ng);
    double Ei, gi;
    if (!GEN || !d.general) {
      Ei = fE[i];
      gi = DIP ? fG[i] : 0.0;
      // P2: the field is linear on the element (fE at its midpoint, slope -h phi_h'')
      if constexpr (P2)
        if (d.order == 2) Ei = Ei - d.h * fG[i] * (frac01(xq, i) - 0.5);
    } else {
      double u;
      general_field(d, fE, fG, i, xq, Q, psi, ps, Ei, gi, u);
      Us += u;
    }
    if constexpr (DIP) {
      if (pend) { P = P + half * Ei; qs = qs + half * ps * gi; }
      Ks += 0.5 * psi * P * P + qs * P;
      Ms += psi * P + qs;
      Cs += psi;
      P = P + half * Ei;
      qs = qs + half * ps * gi;
    } else {
      if (pend) P = P + half * Ei;
      Ks += 0.5 * psi * P * P;
      Ms += psi * P;
      Cs += psi;
      P = P + half * Ei;
    }
    double Qn = Q + dt * P;
    if (Qn < 0.0) Qn += L;
    if (Qn >= L) Qn -= L;
    const T Qs = (T)Qn;
    const double Qd = Qs;
    const double x = Qd * inv_h;
    const int j = cell_of(x, ng);
    const double s = frac01(x, j);
    const bool p2 = P2 && d.order == 2;
    if constexpr (DIP) {
      const double psn = ps - dt * qs;
      const T pss = (T)psn;
      const double psd = pss;
      if (p2) {
        deposit_p2<MODE, true>(sacc, ng, j, s, psi, psd, inv_h);
      } else {
        lds_add<MODE>(sacc, j, psi * (1.0 - s) + psd * inv_h);
        lds_add<MODE>(sacc, (j + 1) & (ng - 1), psi * s - psd * inv_h);
      }
      qsr = (T)qs; psr = pss;
    } else {
      if (p2) {
        deposit_p2<MODE, false>(sacc, ng, j, s, psi, 0.0, inv_h);
      } else {
        lds_add<MODE>(sacc, j, psi * (1.0 - s));
        lds_add<MODE>(sacc, (j + 1) & (ng - 1), psi * s);
      }
    }
    Qr = Qs; Pr = (T)P;
  }
}

// LDS of the fused kernel, in doubles: E [0, Ng), g [Ng, 2Ng), deposit grid [2Ng, 3Ng),
// b~ [3Ng, 4Ng), FFT scratch [4Ng, 7Ng) (FFT solver only).  A P2 instance's deposit grid
// has 2Ng nodes, which moves b~ and the scratch up by Ng: the launch sizes its LDS for
// twice its largest P2 mesh (the `max_ng` of the launch functions).
__host__ __device__ constexpr size_t fused_lds_doubles(bool fft) { return fft ? 7 : 4; }

// One fused step of every tile, in phase r:
//   solve the field of the current positions from ring entry r (every workgroup, redundantly,
//   while its first particle loads are in flight) ->
//   [pending half-kick] -> kinetic sums at the integer step -> half-kick -> drift ->
//   deposit of the drifted state into ring entry r+1.
// The first tile of each instance also records the previous integer step (its kinetic sums
// and field summary are complete once the previous launch ended), stores this step's field
// summary, clears ring entry r+2 and advances the step counter.  No workgroup waits for
// another: the next launch reads what this one deposited.
// Particles per thread whose loads are in flight together (float64 state at 1024 threads
// per workgroup holds two, to stay within 128 registers without spilling).
template <int MODE, int TPB>
__host__ __device__ constexpr int group_of() { return (MODE == kFP64 && TPB == 1024) ? 2 : 4; }

// DIP = false: every tile of the launch belongs to a monopole-only instance; p* and q* are
// neither read nor written (20 bytes of particle traffic per update instead of 36).
// GEN = false: no instance of the launch has general options (d.general), so the field on a
// particle is read straight from the mesh arrays.  P2 = true: the launch's instances have P2
// elements (separate instances keep the others' registers as they were).
template <int MODE, int TPB, bool DIP, bool GEN, bool P2>
__global__ __launch_bounds__(TPB) void k_fused(const InstDev* __restrict__ insts,
                                               const Tile* __restrict__ tiles, int tile0,
                                               int ppt, int phase) {
  extern __shared__ double smem[];
  __shared__ double red[4 * (TPB / 64)];
  __shared__ double sred[kSolveRed];
  using T = typename StateType<MODE>::T;
  constexpr int kGroup = group_of<MODE, TPB>();
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  const int r0 = phase, r1 = ring_next(phase), r2 = ring_prev(phase);
  VPG T* __restrict__ Qp = gp<T>(d.Q);
  VPG T* __restrict__ Pp = gp<T>(d.P);
  VPG T* __restrict__ qsp = gp<T>(d.qs);
  VPG T* __restrict__ psp = gp<T>(d.ps);
  const VPG T* __restrict__ psip = gp<T>(d.psi);
  const int nacc = P2 ? d.nacc : ng;  // load-vector nodes (2 ng for P2)
  double* fE = smem;
  double* fG = smem + ng;
  double* sacc = smem + 2 * ng;
  double* bt = sacc + nacc;
  double* fft = bt + ng;
  VPG InstScal* sc = gp(d.scal);
  // An instance whose diagnostics went NaN / Inf is frozen: its state is no longer a
  // solution, and its particles would all land in element 0.  (Uniform per workgroup.)  The
  // flag is tested once the first loads are out, so its latency overlaps theirs.
  const int frozen = sc->nonfinite;
  const bool first = tl.local == 0;  // the instance's bookkeeping tile (uniform per workgroup)

  // one group of particles per thread: thread t takes tile.begin + k * TPB + t, k0 <= k < k0 + kGroup
  struct Group {
    T q[kGroup], p[kGroup], a[kGroup], b[kGroup], w[kGroup];
    long long idx[kGroup];
    bool v[kGroup];
  };
  auto load_group = [&](int k0, Group& g) {
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int loc = (k0 + u) * TPB + (int)threadIdx.x;
      g.v[u] = (k0 + u < ppt) && (loc < tl.count);
      g.idx[u] = tl.begin + loc;
      if (g.v[u]) {
        g.q[u] = ntld(Qp + g.idx[u]); g.p[u] = ntld(Pp + g.idx[u]); g.w[u] = ntld(psip + g.idx[u]);
        if constexpr (DIP) {
          g.a[u] = ntld(qsp + g.idx[u]); g.b[u] = ntld(psp + g.idx[u]);
        } else {
          g.a[u] = T(0); g.b[u] = T(0);
        }
      }
    }
  };

  // The solve's loads go out first and the first group's particle loads right behind them:
  // both latencies overlap, and the solve can start once its own loads are back (the loads
  // return in order) while the particle loads are still in flight.
  SolveIn sin_;
  solve_load<MODE, false, GEN, P2>(d, r0, first, sin_);
  Group g;
  load_group(0, g);
  if (frozen) return;
  for (int j = threadIdx.x; j < nacc; j += TPB) sacc[j] = 0.0;
  const int pend = sc->pend[r0];
  // the first tile records the previous step (if it was a fused step of this instance):
  // its inputs are read now and written after the solve
  long long step = 0;
  double rec[3] = {0.0, 0.0, 0.0};
  if (first) {
    step = sc->step;
    rec[0] = sc->W[r2];
    rec[1] = sc->e1r[r2];
    rec[2] = sc->e1i[r2];
  }
  double Ks = 0.0, Ms = 0.0, Cs = 0.0, Us = 0.0;
  {
    double sum[7];
    solve_compute<TPB, GEN, P2>(d, sin_, first, bt, fE, fG, sred, fft, nullptr, sum);
    if (first) {
      const int copies = d.acc_copies;
      for (int c = 0; c < copies; ++c)
        for (int j = threadIdx.x; j < nacc; j += TPB) {
          if constexpr (MODE == kFP32)
            gp<float>(d.acc)[acc_off(d, r2, c) + j] = 0.0f;
          else
            gp(d.acc)[acc_off(d, r2, c) + j] = 0.0;
        }
      if (threadIdx.x == 0) {
        if (pend && step >= 1)
          write_record(d, step - 1, sum[3], sum[4], sum[5], sum[6], rec[0], rec[1], rec[2]);
        sc->W[r0] = sum[0];
        sc->e1r[r0] = sum[1];
        sc->e1i[r0] = sum[2];
        if (!isfinite(sum[0])) sc->nonfinite = 1;
        sc->pend[r1] = 1;
        sc->step = step + 1;
      }
    }
  }

  auto run_group = [&](Group& g) {
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      if (!g.v[u]) continue;
      T Q = g.q[u], P = g.p[u], qs = g.a[u], ps = g.b[u];
      push_particle<MODE, T, DIP, GEN, P2>(d, fE, fG, sacc, pend, Q, P, qs, ps, g.w[u], Ks, Ms,
                                           Cs, Us);
      ntst(Qp + g.idx[u], Q); ntst(Pp + g.idx[u], P);
      if constexpr (DIP) { ntst(qsp + g.idx[u], qs); ntst(psp + g.idx[u], ps); }
    }
  };

  run_group(g);
  for (int k0 = kGroup; k0 < ppt; k0 += kGroup) {
    load_group(k0, g);
    run_group(g);
  }

  // kinetic sums: wave trees, one barrier, one thread stores the workgroup totals in this
  // tile's slot (the next pass's first tile adds the slots in tile order)
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  Ks = wave_sum(Ks);
  Ms = wave_sum(Ms);
  Cs = wave_sum(Cs);
  if constexpr (GEN) Us = wave_sum(Us);
  if (lane == 0) {
    red[4 * wid] = Ks;
    red[4 * wid + 1] = Ms;
    red[4 * wid + 2] = Cs;
    if constexpr (GEN) red[4 * wid + 3] = Us;
  }
  __syncthreads();  // also completes every LDS deposit of the workgroup
  if (threadIdx.x == 0) {
    double kb = 0.0, mb = 0.0, cbs = 0.0, ub = 0.0;
    for (int w = 0; w < TPB / 64; ++w) {
      kb += red[4 * w];
      mb += red[4 * w + 1];
      cbs += red[4 * w + 2];
      if constexpr (GEN) ub += red[4 * w + 3];
    }
    VPG double* slot = gp(d.kin) + ((size_t)r0 * d.kin_cap + tl.local) * kKinFields;
    slot[0] = kb;
    slot[1] = mb;
    slot[2] = cbs;
    if constexpr (GEN) slot[3] = ub;  // else it stays zero (no potential in this instance)
  }
  flush<MODE, TPB>(d, sacc, r1, tl.local % d.acc_copies);
}


// ------------------------------------------------------------------ persistent step
// nsteps fused steps in one cooperative launch (every workgroup resident at once).  The
// particles of each tile stay in registers from the first step to the last.  Between steps
// every workgroup of an instance waits until all of the instance's tiles have flushed the
// previous step: an arrival counter, polled by one thread with a bounded spin (after
// kSpinLimit polls the instance is flagged and the wait ends, so every wave finishes).  Data
// other workgroups of the launch wrote (the load vector, the per-tile kinetic sums, the
// cleared ring entry) is read and written at device scope; the ring protocol, the records
// and the arithmetic are those of k_fused, so nsteps persistent steps equal nsteps fused
// launches.  P2 instances are not taken (the host refuses persistent tuning for them).
constexpr unsigned kSpinLimit = 1u << 22;

template <int MODE, int TPB, int PPT>
__global__ __launch_bounds__(TPB) void k_persist(const InstDev* __restrict__ insts,
                                                 const Tile* __restrict__ tiles, int phase0,
                                                 int nsteps) {
  extern __shared__ double smem[];
  __shared__ double red[4 * (TPB / 64)];
  __shared__ double sred[kSolveRed];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  VPG T* __restrict__ Qp = gp<T>(d.Q);
  VPG T* __restrict__ Pp = gp<T>(d.P);
  VPG T* __restrict__ qsp = gp<T>(d.qs);
  VPG T* __restrict__ psp = gp<T>(d.ps);
  const VPG T* __restrict__ psip = gp<T>(d.psi);
  double* fE = smem;
  double* fG = smem + ng;
  double* sacc = smem + 2 * ng;
  double* bt = smem + 3 * ng;
  double* fft = smem + 4 * ng;
  VPG InstScal* sc = gp(d.scal);
  if (sc->frozen) return;  // fixed for the launch: all tiles of the instance leave together
  const bool first = tl.local == 0;

  T q[PPT], p[PPT], a[PPT], b[PPT], w[PPT];
  bool v[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int loc = u * TPB + (int)threadIdx.x;
    v[u] = loc < tl.count;
    if (v[u]) {
      const long long i = tl.begin + loc;
      q[u] = ntld(Qp + i); p[u] = ntld(Pp + i); a[u] = ntld(qsp + i);
      b[u] = ntld(psp + i); w[u] = ntld(psip + i);
    }
  }
  int pend = sc->pend[phase0];
  long long step = 0;
  double rec[3] = {0.0, 0.0, 0.0};  // field summary of the previous step (first tile)
  if (first) {
    step = sc->step;
    rec[0] = sc->W[ring_prev(phase0)];
    rec[1] = sc->e1r[ring_prev(phase0)];
    rec[2] = sc->e1i[ring_prev(phase0)];
  }
  VPG unsigned* arrive = &sc->arrive;

  int r0 = phase0;
  for (int st = 0; st < nsteps; ++st) {
    // nothing is hoisted out of the step loop: keeps the step's registers per step
    __asm__ __volatile__("" ::: "memory");
    const int r1 = ring_next(r0), r2 = ring_prev(r0);
    if (st > 0) {  // wait for every tile of the instance to finish the previous step
      if (threadIdx.x == 0) {
        const unsigned target = (unsigned)st * (unsigned)d.ntiles;
        unsigned it = 0;
        while (__hip_atomic_load(arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
          __builtin_amdgcn_s_sleep(1);
          if (++it > kSpinLimit) {
            __hip_atomic_store(&sc->timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
      __syncthreads();
    }
    SolveIn sin_;
    solve_load<MODE, true, true, false>(d, r0, first, sin_);
    for (int j = threadIdx.x; j < ng; j += TPB) sacc[j] = 0.0;
    double Ks = 0.0, Ms = 0.0, Cs = 0.0, Us = 0.0;
    {
      double sum[7];
      solve_compute<TPB, true, false>(d, sin_, first, bt, fE, fG, sred, fft, nullptr, sum);
      if (first) {
        const int copies = d.acc_copies;
        for (int c = 0; c < copies; ++c)
          for (int j = threadIdx.x; j < ng; j += TPB) {
            if constexpr (MODE == kFP32)
              gst(gp<float>(d.acc) + acc_off(d, r2, c) + j, 0.0f);
            else
              gst(gp(d.acc) + acc_off(d, r2, c) + j, 0.0);
          }
        if (threadIdx.x == 0) {
          if (pend && step >= 1)
            write_record(d, step - 1, sum[3], sum[4], sum[5], sum[6], rec[0], rec[1], rec[2]);
          sc->W[r0] = sum[0];
          sc->e1r[r0] = sum[1];
          sc->e1i[r0] = sum[2];
          if (!isfinite(sum[0])) sc->nonfinite = 1;
          sc->pend[r1] = 1;
          sc->step = step + 1;
        }
        step += 1;
        rec[0] = sum[0];
        rec[1] = sum[1];
        rec[2] = sum[2];
      }
    }
#pragma unroll
    for (int u = 0; u < PPT; ++u)
      if (v[u])
        push_particle<MODE, T, true, true, false>(d, fE, fG, sacc, pend, q[u], p[u], a[u], b[u],
                                                  w[u], Ks, Ms, Cs, Us);
    pend = 1;

    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    Ks = wave_sum(Ks);
    Ms = wave_sum(Ms);
    Cs = wave_sum(Cs);
    Us = wave_sum(Us);
    if (lane == 0) {
      red[4 * wid] = Ks;
      red[4 * wid + 1] = Ms;
      red[4 * wid + 2] = Cs;
      red[4 * wid + 3] = Us;
    }
    __syncthreads();  // also completes every LDS deposit of the workgroup
    if (threadIdx.x == 0) {
      double kb = 0.0, mb = 0.0, cbs = 0.0, ub = 0.0;
      for (int ww = 0; ww < TPB / 64; ++ww) {
        kb += red[4 * ww];
        mb += red[4 * ww + 1];
        cbs += red[4 * ww + 2];
        ub += red[4 * ww + 3];
      }
      VPG double* slot = gp(d.kin) + ((size_t)r0 * d.kin_cap + tl.local) * kKinFields;
      gst(slot, kb);
      gst(slot + 1, mb);
      gst(slot + 2, cbs);
      gst(slot + 3, ub);
    }
    flush<MODE, TPB>(d, sacc, r1, tl.local % d.acc_copies);
    if (st + 1 < nsteps) {
      __builtin_amdgcn_s_waitcnt(0);  // this wave's flush, slot and clear are performed
      __syncthreads();
      if (threadIdx.x == 0)
        __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    r0 = r1;
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u)
    if (v[u]) {
      const long long i = tl.begin + u * TPB + (int)threadIdx.x;
      ntst(Qp + i, q[u]); ntst(Pp + i, p[u]); ntst(qsp + i, a[u]); ntst(psp + i, b[u]);
    }
}

// Deposit of the current state only (eq. rhs-assembly), added into ring entry `phase`.
template <int MODE, int TPB>
__global__ __launch_bounds__(TPB) void k_deposit(const InstDev* __restrict__ insts,
                                                 const Tile* __restrict__ tiles, int tile0,
                                                 int ppt, int phase) {
  extern __shared__ double smem[];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  double* sacc = smem + 2 * ng;
  stage<MODE, TPB>(d, smem, sacc, false, true);
  const VPG T* __restrict__ Qp = gp<T>(d.Q);
  const VPG T* __restrict__ psp = gp<T>(d.ps);
  const VPG T* __restrict__ psip = gp<T>(d.psi);
  if constexpr (MODE == kFP32) {
    const float ihf = (float)d.inv_h;
    float* fa = reinterpret_cast<float*>(sacc);
    VP_TILE_LOOP_BEGIN
    float q[4], b[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) { q[u] = Qp[idx[u]]; b[u] = psp[idx[u]]; w[u] = psip[idx[u]]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const float x = q[u] * ihf;
      const int j = cell_of_f(x, ng);
      const float s = frac01_f(x, j);
      atomicAdd(fa + j, w[u] * (1.0f - s) + b[u] * ihf);
      atomicAdd(fa + ((j + 1) & (ng - 1)), w[u] * s - b[u] * ihf);
    }
    VP_TILE_LOOP_END
  } else {
    const double inv_h = d.inv_h;
    const bool p2 = d.order == 2;
    VP_TILE_LOOP_BEGIN
    T q[4], b[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) { q[u] = Qp[idx[u]]; b[u] = psp[idx[u]]; w[u] = psip[idx[u]]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const double psi = w[u], psd = b[u];
      const double x = (double)q[u] * inv_h;
      const int j = cell_of(x, ng);
      const double s = frac01(x, j);
      if (p2) {
        deposit_p2<MODE, true>(sacc, ng, j, s, psi, psd, inv_h);
      } else {
        lds_add<MODE>(sacc, j, psi * (1.0 - s) + psd * inv_h);
        lds_add<MODE>(sacc, (j + 1) & (ng - 1), psi * s - psd * inv_h);
      }
    }
    VP_TILE_LOOP_END
  }
  __syncthreads();
  flush<MODE, TPB>(d, sacc, phase, tl.local % d.acc_copies);
}

// Kick by `kick` then drift by `drift` with the field arrays.  With use_pending, the kick of
// each instance is dt/2 when its half-kick is pending in phase `phase` and 0 otherwise, and
// drift is 0.
template <int MODE, int TPB>
__global__ __launch_bounds__(TPB) void k_gather_push(const InstDev* __restrict__ insts,
                                                     const Tile* __restrict__ tiles, int tile0,
                                                     int ppt, double kick_in, double drift_in,
                                                     int use_pending, int phase) {
  extern __shared__ double smem[];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  double kick = kick_in, drift = drift_in;
  if (use_pending) {
    kick = gp(d.scal)->pend[phase] ? 0.5 * d.dt : 0.0;
    drift = 0.0;
  }
  if (kick == 0.0 && drift == 0.0) return;  // uniform per workgroup: no barrier skipped
  stage<MODE, TPB>(d, smem, nullptr, true, false);
  VPG T* __restrict__ Qp = gp<T>(d.Q);
  VPG T* __restrict__ Pp = gp<T>(d.P);
  VPG T* __restrict__ qsp = gp<T>(d.qs);
  VPG T* __restrict__ psp = gp<T>(d.ps);
  const bool do_kick = kick != 0.0, do_drift = drift != 0.0;
  if constexpr (MODE == kFP32) {
    const float* fE = reinterpret_cast<const float*>(smem);
    const float* fG = fE + ng;
    const float Lf = (float)d.L, ihf = (float)d.inv_h, kf = (float)kick, df = (float)drift;
    VP_TILE_LOOP_BEGIN
    float q[4], p[4], a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) { q[u] = Qp[idx[u]]; p[u] = Pp[idx[u]]; a[u] = qsp[idx[u]]; b[u] = psp[idx[u]]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      float Q = q[u], P = p[u], qs = a[u], ps = b[u];
      const float xq = Q * ihf;
      const int i = cell_of_f(xq, ng);
      float Ei, gi;
      if (!d.general) {
        Ei = fE[i];
        gi = fG[i];
      } else {
        double e, g, uu;
        general_field(d, fE, fG, i, (double)Q * d.inv_h, (double)Q, 0.0, 0.0, e, g, uu);
        Ei = (float)e;
        gi = (float)g;
      }
      P = P + kf * Ei;
      qs = qs + kf * ps * gi;
      float Qn = Q + df * P;
      if (Qn < 0.0f) Qn += Lf;
      if (Qn >= Lf) Qn -= Lf;
      ps = ps - df * qs;
      if (do_kick) { Pp[idx[u]] = P; qsp[idx[u]] = qs; }
      if (do_drift) { Qp[idx[u]] = Qn; psp[idx[u]] = ps; }
    }
    VP_TILE_LOOP_END
  } else {
    const double L = d.L, inv_h = d.inv_h;
    VP_TILE_LOOP_BEGIN
    T q[4], p[4], a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) { q[u] = Qp[idx[u]]; p[u] = Pp[idx[u]]; a[u] = qsp[idx[u]]; b[u] = psp[idx[u]]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const double Q = q[u];
      double P = p[u], qs = a[u], ps = b[u];
      const double xq = Q * inv_h;
      const int i = cell_of(xq, ng);
      double Ei, gi;
      if (!d.general) {
        Ei = smem[i];
        gi = smem[ng + i];
        if (d.order == 2) Ei = Ei - d.h * gi * (frac01(xq, i) - 0.5);  // P2: linear field
      } else {
        double uu;
        general_field(d, smem, smem + ng, i, xq, (double)Q, 0.0, 0.0, Ei, gi, uu);
      }
      P = P + kick * Ei;
      qs = qs + kick * ps * gi;
      double Qn = Q + drift * P;
      if (Qn < 0.0) Qn += L;
      if (Qn >= L) Qn -= L;
      ps = ps - drift * qs;
      if (do_kick) { Pp[idx[u]] = (T)P; qsp[idx[u]] = (T)qs; }
      if (do_drift) { Qp[idx[u]] = (T)Qn; psp[idx[u]] = (T)ps; }
    }
    VP_TILE_LOOP_END
  }
}

// Kinetic diagnostics at the integer step without touching the state: a pending half-kick
// is applied to local copies only.
template <int MODE, int TPB>
__global__ __launch_bounds__(TPB) void k_diag(const InstDev* __restrict__ insts,
                                              const Tile* __restrict__ tiles, int tile0,
                                              int ppt, int phase) {
  extern __shared__ double smem[];
  __shared__ double red[TPB / 64];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  stage<MODE, TPB>(d, smem, nullptr, true, false);
  const VPG T* __restrict__ Qp = gp<T>(d.Q);
  const VPG T* __restrict__ Pp = gp<T>(d.P);
  const VPG T* __restrict__ qsp = gp<T>(d.qs);
  const VPG T* __restrict__ psp = gp<T>(d.ps);
  const VPG T* __restrict__ psip = gp<T>(d.psi);
  const int pend = gp(d.scal)->pend[phase];
  double Ks = 0.0, Ms = 0.0, Cs = 0.0, Us = 0.0;
  if constexpr (MODE == kFP32) {
    const float* fE = reinterpret_cast<const float*>(smem);
    const float* fG = fE + ng;
    const float ihf = (float)d.inv_h, hf = 0.5f * (float)d.dt;
    VP_TILE_LOOP_BEGIN
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const float Q = Qp[idx[u]], psi = psip[idx[u]], ps = psp[idx[u]];
      float P = Pp[idx[u]], qs = qsp[idx[u]];
      const float xq = Q * ihf;
      const int i = cell_of_f(xq, ng);
      float Ei, gi;
      if (!d.general) {
        Ei = fE[i];
        gi = fG[i];
      } else {
        double e, g, uu;
        general_field(d, fE, fG, i, (double)Q * d.inv_h, (double)Q, (double)psi, (double)ps, e,
                      g, uu);
        Ei = (float)e;
        gi = (float)g;
        Us += uu;
      }
      if (pend) {
        P = P + hf * Ei;
        qs = qs + hf * ps * gi;
      }
      const double Pd = P, qd = qs, wd = psi;
      Ks += 0.5 * wd * Pd * Pd + qd * Pd;
      Ms += wd * Pd + qd;
      Cs += wd;
    }
    VP_TILE_LOOP_END
  } else {
    const double inv_h = d.inv_h, half = 0.5 * d.dt;
    VP_TILE_LOOP_BEGIN
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const double Q = Qp[idx[u]], psi = psip[idx[u]], ps = psp[idx[u]];
      double P = Pp[idx[u]], qs = qsp[idx[u]];
      const double xq = Q * inv_h;
      const int i = cell_of(xq, ng);
      double Ei, gi;
      if (!d.general) {
        Ei = smem[i];
        gi = smem[ng + i];
        if (d.order == 2) Ei = Ei - d.h * gi * (frac01(xq, i) - 0.5);  // P2: linear field
      } else {
        double uu;
        general_field(d, smem, smem + ng, i, xq, Q, psi, ps, Ei, gi, uu);
        Us += uu;
      }
      if (pend) {
        P = P + half * Ei;
        qs = qs + half * ps * gi;
      }
      Ks += 0.5 * psi * P * P + qs * P;
      Ms += psi * P + qs;
      Cs += psi;
    }
    VP_TILE_LOOP_END
  }
  const double Kb = block_sum<TPB>(Ks, red);
  const double Mb = block_sum<TPB>(Ms, red);
  const double Cb = block_sum<TPB>(Cs, red);
  const double Ub = block_sum<TPB>(Us, red);
  if (threadIdx.x == 0) {
    VPG InstScal* sc = gp(d.scal);
    gadd(&sc->Kd, Kb);
    gadd(&sc->momd, Mb);
    gadd(&sc->chgd, Cb);
    gadd(&sc->Ud, Ub);
  }
}

// One workgroup per listed slot: solve the field of ring entry `phase` and write the field
// arrays and the field summary (materialise); when the instance's last pass was a fused
// step, also write that step's record (the next fused pass would write the same record).
template <int MODE>
__global__ __launch_bounds__(kSolveThreads) void k_solve(const InstDev* __restrict__ insts,
                                                         const int* __restrict__ slots,
                                                         int phase) {
  extern __shared__ double smem[];
  __shared__ double sred[kSolveRed];
  const InstDev& d = insts[slots[blockIdx.x]];
  const int ng = d.ng;
  const bool p2 = d.order == 2;
  double* fE = smem;
  double* fG = smem + ng;
  double* phi = smem + 2 * ng;
  double* bt = smem + 3 * ng;
  double* fft = smem + 4 * ng;
  // P2: b~ of vertices and midpoints, after the FFT scratch when this instance uses it
  double* p2b = smem + (d.solver == VP_SOLVE_FFT ? 7 : 4) * ng;
  SolveIn sin_;
  solve_load<MODE>(d, phase, true, sin_);
  double sum[7];
  solve_compute<kSolveThreads>(d, sin_, true, bt, fE, fG, sred, fft, phi, sum,
                               p2 ? p2b : nullptr);
  VPG double* bt_g = gp(d.bt);
  VPG double* E_g = gp(d.E);
  VPG double* g_g = gp(d.g);
  VPG double* Phi_g = gp(d.Phi);
  VPG float* Ef_g = gp(d.Ef);
  VPG float* gf_g = gp(d.gf);
  if (!p2) {
    for (int e = threadIdx.x; e < ng; e += kSolveThreads) {
      const double Ee = fE[e], ge = fG[e];
      bt_g[e] = bt[e];
      E_g[e] = Ee;
      Ef_g[e] = (float)Ee;
      g_g[e] = ge;
      gf_g[e] = (float)ge;
      Phi_g[e] = phi[e];
    }
  } else {
    // midpoint potentials from their own rows, Phi_m = (3h b~_m + 8 (Phi_e + Phi_{e+1})) / 16;
    // then the P2 gauge: shift by c so that (h/3) sum Phi_v + (2h/3) sum Phi_m = 0
    const int per = solve_per(ng);
    double pm[kSolvePer];
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < kSolvePer; ++k) {
      pm[k] = 0.0;
      const int e = threadIdx.x * per + k;
      if (k < per && e < ng) {
        pm[k] = (3.0 * d.h * p2b[ng + e] + 8.0 * (phi[e] + phi[(e + 1) & (ng - 1)])) / 16.0;
        part += phi[e] + 2.0 * pm[k];
      }
    }
    const double c = -block_sum<kSolveThreads>(part, sred) / (3.0 * (double)ng);
#pragma unroll
    for (int k = 0; k < kSolvePer; ++k) {
      const int e = threadIdx.x * per + k;
      if (k < per && e < ng) {
        bt_g[e] = p2b[e];
        bt_g[ng + e] = p2b[ng + e];
        Phi_g[e] = phi[e] + c;
        Phi_g[ng + e] = pm[k] + c;
      }
    }
    for (int e = threadIdx.x; e < ng; e += kSolveThreads) {
      const double Ee = fE[e], ge = fG[e];
      E_g[e] = Ee;
      Ef_g[e] = (float)Ee;
      g_g[e] = ge;
      gf_g[e] = (float)ge;
    }
  }
  if (threadIdx.x == 0) {
    VPG InstScal* sc = gp(d.scal);
    const int r2 = ring_prev(phase);
    if (sc->pend[phase] && sc->step >= 1)
      write_record(d, sc->step - 1, sum[3], sum[4], sum[5], sum[6], sc->W[r2], sc->e1r[r2],
                   sc->e1i[r2]);
    sc->W[phase] = sum[0];
    sc->e1r[phase] = sum[1];
    sc->e1i[phase] = sum[2];
    if (!isfinite(sum[0])) sc->nonfinite = 1;
  }
}

// Ring maintenance, one workgroup per listed slot (see RingOp).
template <typename A>
__global__ __launch_bounds__(256) void k_ring(const InstDev* __restrict__ insts,
                                              const int* __restrict__ slots, int op, int phase) {
  const InstDev& d = insts[slots[blockIdx.x]];
  const int nacc = d.nacc;
  VPG A* acc = gp<A>(reinterpret_cast<A*>(d.acc));
  for (int j = threadIdx.x; j < nacc; j += 256) {
    if (op == kRingFold) {
      double s = 0.0;
      for (int c = 0; c < VP_MAX_ACC_COPIES; ++c) s += (double)acc[acc_off(d, phase, c) + j];
      acc[acc_off(d, phase, 0) + j] = (A)s;
      for (int c = 1; c < VP_MAX_ACC_COPIES; ++c) acc[acc_off(d, phase, c) + j] = (A)0;
      for (int c = 0; c < VP_MAX_ACC_COPIES; ++c) {
        acc[acc_off(d, ring_next(phase), c) + j] = (A)0;
        acc[acc_off(d, ring_prev(phase), c) + j] = (A)0;
      }
    } else {
      for (int c = 0; c < VP_MAX_ACC_COPIES; ++c) acc[acc_off(d, phase, c) + j] = (A)0;
    }
  }
  if (op == kRingFold) {
    // per-tile kinetic sums: the tile count may change, so each entry's sum moves to tile 0
    // and the other tiles are cleared.  Thread t adds tiles t, t + 256, ... in order, then
    // thread 0 adds the 256 partial sums in thread order (fixed order, deterministic).
    __shared__ double part[256];
    VPG double* kin = gp(d.kin);
    for (int rf = 0; rf < kRing * kKinFields; ++rf) {
      const int r = rf / kKinFields, f = rf % kKinFields;
      VPG double* base = kin + (size_t)r * d.kin_cap * kKinFields + f;
      double acc_t = 0.0;
      for (int t = threadIdx.x; t < d.kin_cap; t += 256) acc_t += base[(size_t)t * kKinFields];
      __syncthreads();
      part[threadIdx.x] = acc_t;
      __syncthreads();
      for (int t = threadIdx.x; t < d.kin_cap; t += 256) base[(size_t)t * kKinFields] = 0.0;
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < 256; ++t) s += part[t];
        base[0] = s;
      }
    }
  }
}

__global__ void k_slot_scalars(const InstDev* __restrict__ insts, const int* __restrict__ slots,
                               int nslots, int op, int phase) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  VPG InstScal* sc = gp(insts[slots[t]].scal);
  if (op == kScalClearDiag) {
    sc->Kd = 0.0;
    sc->Ud = 0.0;
    sc->momd = 0.0;
    sc->chgd = 0.0;
  } else if (op == kScalClearPending) {
    sc->pend[phase] = 0;
  } else if (op == kScalPersistStart) {
    sc->frozen = sc->nonfinite;
    sc->arrive = 0u;
  }
}

__global__ void k_slot_status(const InstDev* __restrict__ insts, const int* __restrict__ slots,
                              int nslots, long long* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  const VPG InstScal* sc = gp(insts[slots[t]].scal);
  out[2 * t] = sc->step;
  out[2 * t + 1] = sc->nonfinite;
}

// Zero n8 64-bit words, then a trailing 32-bit word when tail4 (an odd count of floats).
__global__ void k_fill_zero(unsigned long long* p, size_t n8, bool tail4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t i = t; i < n8; i += stride) p[i] = 0ull;
  if (tail4 && t == 0) reinterpret_cast<unsigned*>(p + n8)[0] = 0u;
}

template <typename T>
__global__ void k_cell_index(const InstDev* __restrict__ insts, int slot, int* __restrict__ cells,
                             long long n) {
  const InstDev& d = insts[slot];
  const VPG T* Qp = gp<T>(d.Q);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    cells[k] = cell_of((double)Qp[k] * d.inv_h, d.ng);
}

// ------------------------------------------------------------------ chunked stable sort
// Workgroup b sorts particles [b*chunk, min(n, (b+1)*chunk)) by cell (float64 index
// formula) with two stable 5-bit counting passes in LDS, then permutes the five arrays
// in place through an LDS staging buffer.
template <typename T>
__device__ void permute_array(VPG T* __restrict__ X, long long c0, int m, const unsigned short* order,
                              T* stagebuf) {
  for (int k = threadIdx.x; k < m; k += kBlock) stagebuf[k] = X[c0 + order[k]];
  __syncthreads();
  for (int k = threadIdx.x; k < m; k += kBlock) X[c0 + k] = stagebuf[k];
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sort(const InstDev* __restrict__ insts, int slot,
                                                 long long n, int chunk, int* __restrict__ perm) {
  extern __shared__ double smem[];
  __shared__ int wtot[4];
  const InstDev& d = insts[slot];
  const long long c0 = (long long)blockIdx.x * chunk;
  const long long rem = n - c0;
  const int m = (int)(rem < (long long)chunk ? rem : (long long)chunk);
  T* stagebuf = reinterpret_cast<T*>(smem);                                   // chunk T
  unsigned short* kA = reinterpret_cast<unsigned short*>(stagebuf + chunk);   // 4 x chunk
  unsigned short* kB = kA + chunk;
  unsigned short* iA = kB + chunk;
  unsigned short* iB = iA + chunk;
  int* cnt = reinterpret_cast<int*>(iB + chunk);                              // 32 x 256
  const int tid = threadIdx.x;
  const VPG T* Qp = gp<T>(d.Q);
  for (int k = tid; k < m; k += kBlock) {
    kA[k] = (unsigned short)cell_of((double)Qp[c0 + k] * d.inv_h, d.ng);
    iA[k] = (unsigned short)k;
  }
  __syncthreads();
  const int seg = (m + kBlock - 1) / kBlock;
  const int lo = min(m, tid * seg), hi = min(m, lo + seg);
  for (int pass = 0; pass < 2; ++pass) {
    const int shift = 5 * pass;
    const unsigned short* sk = pass ? kB : kA;
    const unsigned short* si = pass ? iB : iA;
    unsigned short* dk = pass ? kA : kB;
    unsigned short* di = pass ? iA : iB;
    for (int bkt = 0; bkt < 32; ++bkt) cnt[bkt * kBlock + tid] = 0;
    for (int k = lo; k < hi; ++k) cnt[((sk[k] >> shift) & 31) * kBlock + tid] += 1;
    __syncthreads();
    int running = 0;
    for (int bkt = 0; bkt < 32; ++bkt) {
      const int val = cnt[bkt * kBlock + tid];
      int incl = val;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if ((tid & 63) >= off) incl += y;
      }
      if ((tid & 63) == 63) wtot[tid >> 6] = incl;
      __syncthreads();
      int before = 0;
      for (int w = 0; w < (tid >> 6); ++w) before += wtot[w];
      const int total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
      cnt[bkt * kBlock + tid] = running + before + incl - val;
      running += total;
      __syncthreads();
    }
    for (int k = lo; k < hi; ++k) {
      const int bkt = (sk[k] >> shift) & 31;
      const int pos = cnt[bkt * kBlock + tid]++;
      dk[pos] = sk[k];
      di[pos] = si[k];
    }
    __syncthreads();
  }
  if (perm)
    for (int k = tid; k < m; k += kBlock) perm[c0 + k] = (int)(c0 + iA[k]);
  permute_array<T>(gp<T>(d.Q), c0, m, iA, stagebuf);
  permute_array<T>(gp<T>(d.P), c0, m, iA, stagebuf);
  permute_array<T>(gp<T>(d.qs), c0, m, iA, stagebuf);
  permute_array<T>(gp<T>(d.ps), c0, m, iA, stagebuf);
  permute_array<T>(gp<T>(d.psi), c0, m, iA, stagebuf);
}

// ------------------------------------------------------------------ host launchers
static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

WsLayout workspace_layout(int ng, int order, int hist_cap, long long n) {
  WsLayout w{};
  size_t o = 0;
  const size_t nacc = (size_t)(order == 2 ? 2 : 1) * ng;
  w.acc = o;     o = align256(o + (size_t)kRing * VP_MAX_ACC_COPIES * nacc * sizeof(double));
  w.E = o;       o = align256(o + (size_t)ng * sizeof(double));
  w.g = o;       o = align256(o + (size_t)ng * sizeof(double));
  w.Ef = o;      o = align256(o + (size_t)ng * sizeof(float));
  w.gf = o;      o = align256(o + (size_t)ng * sizeof(float));
  w.Phi = o;     o = align256(o + nacc * sizeof(double));
  w.bt = o;      o = align256(o + nacc * sizeof(double));
  w.tw = o;      o = align256(o + (size_t)ng * sizeof(double));
  w.inv_lam = o; o = align256(o + (size_t)ng * sizeof(double));
  w.cw = o;      o = align256(o + (size_t)kConsTapsMax * sizeof(double));
  w.scal = o;    o = align256(o + sizeof(InstScal));
  w.hist = o;    o = align256(o + (size_t)hist_cap * kHistFields * sizeof(double));
  w.kin = o;     o = align256(o + (size_t)kRing * kin_capacity(n) * kKinFields * sizeof(double));
  w.total = o;
  return w;
}

int kin_capacity(long long n) { return (int)((n + kMinTile - 1) / kMinTile); }

size_t particle_lds_bytes(int /*mode*/, int max_ng) {
  return lds_doubles_per_node() * (size_t)max_ng * sizeof(double);
}

#define VP_DISPATCH(mode, tpb, KERNEL, ...)                                                  \
  do {                                                                                       \
    if ((mode) == kFP32TwoSum) {                                                             \
      if ((tpb) == 1024) hipLaunchKernelGGL((KERNEL<kFP32TwoSum, 1024>), __VA_ARGS__);       \
      else if ((tpb) == 512) hipLaunchKernelGGL((KERNEL<kFP32TwoSum, 512>), __VA_ARGS__);    \
      else hipLaunchKernelGGL((KERNEL<kFP32TwoSum, 256>), __VA_ARGS__);                      \
    } else if ((mode) == kFP64) {                                                            \
      if ((tpb) == 1024) hipLaunchKernelGGL((KERNEL<kFP64, 1024>), __VA_ARGS__);             \
      else if ((tpb) == 512) hipLaunchKernelGGL((KERNEL<kFP64, 512>), __VA_ARGS__);          \
      else hipLaunchKernelGGL((KERNEL<kFP64, 256>), __VA_ARGS__);                            \
    } else if ((mode) == kFP32Comp) {                                                        \
      if ((tpb) == 1024) hipLaunchKernelGGL((KERNEL<kFP32Comp, 1024>), __VA_ARGS__);         \
      else if ((tpb) == 512) hipLaunchKernelGGL((KERNEL<kFP32Comp, 512>), __VA_ARGS__);      \
      else hipLaunchKernelGGL((KERNEL<kFP32Comp, 256>), __VA_ARGS__);                        \
    } else {                                                                                 \
      if ((tpb) == 1024) hipLaunchKernelGGL((KERNEL<kFP32, 1024>), __VA_ARGS__);             \
      else if ((tpb) == 512) hipLaunchKernelGGL((KERNEL<kFP32, 512>), __VA_ARGS__);          \
      else hipLaunchKernelGGL((KERNEL<kFP32, 256>), __VA_ARGS__);                            \
    }                                                                                        \
  } while (0)

hipError_t launch_fused(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                        int ntiles, int ppt, int max_ng, bool lds_fft, int phase, bool dipoles,
                        bool general, bool p2, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t lds = fused_lds_doubles(lds_fft) * (size_t)max_ng * sizeof(double);
#define VP_FUSED_K(M, TB, D, G, P)                                                           \
  hipLaunchKernelGGL((k_fused<M, TB, D, G, P>), dim3(ntiles), dim3(TB), lds, s, d_inst,      \
                     d_tiles, tile0, ppt, phase)
#define VP_FUSED(M, TB)                                                                      \
  do {                                                                                       \
    if (dipoles) {                                                                           \
      if (p2) {                                                                              \
        if (general) VP_FUSED_K(M, TB, true, true, true);                                    \
        else VP_FUSED_K(M, TB, true, false, true);                                           \
      } else {                                                                               \
        if (general) VP_FUSED_K(M, TB, true, true, false);                                   \
        else VP_FUSED_K(M, TB, true, false, false);                                          \
      }                                                                                      \
    } else {                                                                                 \
      if (p2) {                                                                              \
        if (general) VP_FUSED_K(M, TB, false, true, true);                                   \
        else VP_FUSED_K(M, TB, false, false, true);                                          \
      } else {                                                                               \
        if (general) VP_FUSED_K(M, TB, false, true, false);                                  \
        else VP_FUSED_K(M, TB, false, false, false);                                         \
      }                                                                                      \
    }                                                                                        \
  } while (0)
#define VP_FUSED_TPB(M)                                                                      \
  do {                                                                                       \
    if (tpb == 1024) VP_FUSED(M, 1024);                                                      \
    else if (tpb == 512) VP_FUSED(M, 512);                                                   \
    else VP_FUSED(M, 256);                                                                   \
  } while (0)
  if (mode == kFP32TwoSum) VP_FUSED_TPB(kFP32TwoSum);
  else if (mode == kFP64) VP_FUSED_TPB(kFP64);
  else if (mode == kFP32Comp) VP_FUSED_TPB(kFP32Comp);
  else VP_FUSED_TPB(kFP32);
#undef VP_FUSED_TPB
#undef VP_FUSED
#undef VP_FUSED_K
  return hipGetLastError();
}


#define VP_PERSIST_CASE(M, TB, PP)                                                          \
  if (mode == M && tpb == TB && ppt == PP) {                                                \
    fn = reinterpret_cast<const void*>(&k_persist<M, TB, PP>);                              \
  }

static const void* persist_fn(int mode, int tpb, int ppt) {
  const void* fn = nullptr;
#define VP_PERSIST_MODE(M)                                                                  \
  VP_PERSIST_CASE(M, 512, 2) VP_PERSIST_CASE(M, 512, 4) VP_PERSIST_CASE(M, 512, 8)          \
  VP_PERSIST_CASE(M, 1024, 2) VP_PERSIST_CASE(M, 1024, 4) VP_PERSIST_CASE(M, 1024, 8)
  VP_PERSIST_MODE(kFP64)
  VP_PERSIST_MODE(kFP32Comp)
  VP_PERSIST_MODE(kFP32)
  VP_PERSIST_MODE(kFP32TwoSum)
#undef VP_PERSIST_MODE
  return fn;
}
#undef VP_PERSIST_CASE

int persist_capacity(int mode, int tpb, int ppt, int max_ng, bool lds_fft) {
  const void* fn = persist_fn(mode, tpb, ppt);
  if (!fn) return 0;
  const size_t lds = fused_lds_doubles(lds_fft) * (size_t)max_ng * sizeof(double);
  int per_cu = 0, cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, tpb, lds) != hipSuccess) return 0;
  return per_cu * cus;
}

hipError_t launch_persist(int mode, int tpb, int ppt, const InstDev* d_inst, const Tile* d_tiles,
                          int ntiles, int max_ng, bool lds_fft, int phase, int nsteps,
                          hipStream_t s) {
  if (ntiles <= 0 || nsteps <= 0) return hipSuccess;
  const void* fn = persist_fn(mode, tpb, ppt);
  if (!fn) return hipErrorInvalidValue;
  const size_t lds = fused_lds_doubles(lds_fft) * (size_t)max_ng * sizeof(double);
  void* args[] = {(void*)&d_inst, (void*)&d_tiles, (void*)&phase, (void*)&nsteps};
  return hipLaunchCooperativeKernel(fn, dim3(ntiles), dim3(tpb), args, (unsigned)lds, s);
}

hipError_t launch_deposit(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                          int ntiles, int ppt, int max_ng, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_deposit, dim3(ntiles), dim3(tpb), particle_lds_bytes(mode, max_ng), s,
              d_inst, d_tiles, tile0, ppt, phase);
  return hipGetLastError();
}

hipError_t launch_gather_push(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles,
                              int tile0, int ntiles, int ppt, int max_ng, double kick, double drift,
                              hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_gather_push, dim3(ntiles), dim3(tpb),
              (size_t)2 * max_ng * sizeof(double), s, d_inst, d_tiles, tile0, ppt, kick, drift, 0,
              0);
  return hipGetLastError();
}

hipError_t launch_settle(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                         int ntiles, int ppt, int max_ng, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_gather_push, dim3(ntiles), dim3(tpb),
              (size_t)2 * max_ng * sizeof(double), s, d_inst, d_tiles, tile0, ppt, 0.0, 0.0, 1,
              phase);
  return hipGetLastError();
}

hipError_t launch_diag(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                       int ntiles, int ppt, int max_ng, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_diag, dim3(ntiles), dim3(tpb), (size_t)2 * max_ng * sizeof(double), s,
              d_inst, d_tiles, tile0, ppt, phase);
  return hipGetLastError();
}

hipError_t launch_solve(int mode, const InstDev* d_inst, const int* d_slots, int nslots,
                        int max_ng, bool lds_fft, int phase, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  const size_t lds = fused_lds_doubles(lds_fft) * (size_t)max_ng * sizeof(double);
  if (mode == kFP64 || mode == kFP32TwoSum)
    hipLaunchKernelGGL(k_solve<kFP64>, dim3(nslots), dim3(kSolveThreads), lds, s, d_inst, d_slots,
                       phase);
  else if (mode == kFP32Comp)
    hipLaunchKernelGGL(k_solve<kFP32Comp>, dim3(nslots), dim3(kSolveThreads), lds, s, d_inst,
                       d_slots, phase);
  else
    hipLaunchKernelGGL(k_solve<kFP32>, dim3(nslots), dim3(kSolveThreads), lds, s, d_inst, d_slots,
                       phase);
  return hipGetLastError();
}

hipError_t launch_ring(int mode, const InstDev* d_inst, const int* d_slots, int nslots, int op,
                       int phase, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  if (mode == kFP32)
    hipLaunchKernelGGL(k_ring<float>, dim3(nslots), dim3(256), 0, s, d_inst, d_slots, op, phase);
  else
    hipLaunchKernelGGL(k_ring<double>, dim3(nslots), dim3(256), 0, s, d_inst, d_slots, op, phase);
  return hipGetLastError();
}

hipError_t launch_slot_scalars(const InstDev* d_inst, const int* d_slots, int nslots, int op,
                               int phase, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_scalars, dim3((nslots + 63) / 64), dim3(64), 0, s, d_inst, d_slots,
                     nslots, op, phase);
  return hipGetLastError();
}

hipError_t launch_slot_status(const InstDev* d_inst, const int* d_slots, int nslots,
                              long long* out, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_status, dim3((nslots + 63) / 64), dim3(64), 0, s, d_inst, d_slots,
                     nslots, out);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  // bytes: a multiple of 4 (whole float or double elements)
  const size_t n8 = bytes / 8;
  const bool tail4 = (bytes % 8) >= 4;
  if (n8 == 0 && !tail4) return hipSuccess;
  size_t blocks = (n8 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<unsigned long long*>(p), n8, tail4);
  return hipGetLastError();
}

hipError_t launch_cell_index(const InstDev* d_inst, int slot, int mode, int* cells, long long n,
                             hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (mode == kFP64)
    hipLaunchKernelGGL(k_cell_index<double>, dim3((unsigned)blocks), dim3(256), 0, s, d_inst, slot,
                       cells, n);
  else
    hipLaunchKernelGGL(k_cell_index<float>, dim3((unsigned)blocks), dim3(256), 0, s, d_inst, slot,
                       cells, n);
  return hipGetLastError();
}

hipError_t launch_sort(int mode, const InstDev* d_inst, int slot, long long n, int chunk,
                       int* perm, hipStream_t s) {
  const long long blocks = (n + chunk - 1) / chunk;
  if (blocks <= 0) return hipSuccess;
  const size_t tsz = (mode == kFP64) ? sizeof(double) : sizeof(float);
  const size_t lds = (size_t)chunk * tsz + (size_t)4 * chunk * sizeof(unsigned short) +
                     (size_t)32 * kBlock * sizeof(int);
  if (mode == kFP64)
    hipLaunchKernelGGL(k_sort<double>, dim3((unsigned)blocks), dim3(kBlock), lds, s, d_inst, slot,
                       n, chunk, perm);
  else
    hipLaunchKernelGGL(k_sort<float>, dim3((unsigned)blocks), dim3(kBlock), lds, s, d_inst, slot,
                       n, chunk, perm);
  return hipGetLastError();
}

}  // namespace vpk

// Device-side building blocks shared by the kernel translation units of libvp (gfx950):
// state types, address-space helpers, cell location, the LDS deposit, the flush into the
// global accumulators, the wavefront collectives, the Poisson solve and the per-particle
// step.  Everything here is a template or inline, or static to each unit.
//
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

#pragma once

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

// Element index of x = Q * Ng / L: floor, clamped to [0, Ng-1] (NaN maps to 0: fmax returns
// the number when one operand is NaN), so an LDS index is always in range whatever the state
// holds.  Branch-free, so the particles of one thread interleave.
__device__ __forceinline__ int cell_of(double x, int ng) {
  return (int)fmin(fmax(floor(x), 0.0), (double)(ng - 1));
}
__device__ __forceinline__ int cell_of_f(float x, int ng) {
  return (int)fminf(fmaxf(floorf(x), 0.0f), (float)(ng - 1));
}
// 2^-m exactly (0 <= m <= 1022): x * inv_pow2(m) equals x / 2^m bit for bit, without the
// division's instruction sequence.
__device__ __forceinline__ double inv_pow2(int m) {
  return __longlong_as_double((long long)(1023 - m) << 52);
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

// Deposit of one particle's NV nodal contributions c[k] into nodes node[k] of element j.
// In the compensated float32 mode, with `seg` (vp_tuning.wave_reduce, uniform per
// workgroup), the wavefront first combines the contributions of neighbouring lanes that hit
// the same element: lanes whose left neighbour has the same element continue a run; a
// segmented inclusive sum over each run (Hillis-Steele over lane shuffles, clipped at the
// run's first lane) leaves the run's totals in its last lane, which alone commits them to
// the LDS grid.  Runs arise when particles that are neighbours in memory are neighbours in
// space (sorted by cell, or bunched in a lattice order); when fewer than kSegMin lanes
// continue a run the lanes update the grid one by one, as without `seg`.  The combination
// needs every lane of the wavefront active (checked; otherwise the per-lane updates).  Sums
// differ from the per-lane updates in their order only.  The float64 LDS add takes
// same-node lanes faster than the scan would (measured), so the modes that accumulate in
// float64 always update per lane; the (hi, lo) pairs pay a compare-and-swap per update.
constexpr int kSegMin = 8;
template <int MODE, int NV>
__device__ __forceinline__ void deposit_nodes(double* sacc, bool seg, int j, const int (&node)[NV],
                                              double (&c)[NV]) {
  if (MODE == kFP32TwoSum && seg && __builtin_amdgcn_read_exec() == ~0ull) {
    // element of lane - 1 (lane 0: -1, never an element), by a DPP wavefront shift
    const int jp = __builtin_amdgcn_update_dpp(-1, j, 0x138, 0xf, 0xf, false);
    const unsigned long long cont = __ballot(jp == j);
    if (__popcll(cont) >= kSegMin) {
      const int lane = __lane_id();
      int rs = (jp == j) ? 0 : lane;  // first lane of this lane's run, by a max-scan
      for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(rs, off);
        if (lane >= off) rs = max(rs, t);
      }
      for (int off = 1; off < 64; off <<= 1) {
        double t[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) t[k] = __shfl_up(c[k], off);
        if (lane - off >= rs)
#pragma unroll
          for (int k = 0; k < NV; ++k) c[k] += t[k];
      }
      // element of lane + 1 (lane 63: -1): the run's last lane holds its totals
      const int jn = __builtin_amdgcn_update_dpp(-1, j, 0x130, 0xf, 0xf, false);
      if (jn != j)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds_add<MODE>(sacc, node[k], c[k]);
      return;
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) lds_add<MODE>(sacc, node[k], c[k]);
}

// P2 load of one particle at local coordinate s of element j (eq. galerkin with the
// quadratic basis N0 = (1-s)(1-2s), N1 = 4s(1-s), N2 = s(2s-1) of the element's left vertex,
// midpoint and right vertex): node k gets psi* N_k(s) - p* N_k'(s) / h.  Midpoint j is LDS
// entry ng + j.  With DIP false p* is zero and its terms are left out.
// K3: the particle also carries second moments, and Mqq adds (1/2) Mqq phi_k''(Q): the
// basis' second derivatives on the element are 4, -8, 4 (left vertex, midpoint, right vertex)
// over h^2.
template <int MODE, bool DIP, bool K3 = false>
__device__ __forceinline__ void deposit_p2(double* sacc, int ng, int j, double s, double psi,
                                           double ps, double inv_h, double mqq = 0.0,
                                           bool seg = false) {
  const double n0 = (1.0 - s) * (1.0 - 2.0 * s), n1 = 4.0 * s * (1.0 - s), n2 = s * (2.0 * s - 1.0);
  const int node[3] = {j, ng + j, (j + 1) & (ng - 1)};
  double c[3];
  if constexpr (K3) {
    const double m = 0.5 * mqq * (inv_h * inv_h);
    c[0] = psi * n0 - ps * ((4.0 * s - 3.0) * inv_h) + 4.0 * m;
    c[1] = psi * n1 - ps * ((4.0 - 8.0 * s) * inv_h) - 8.0 * m;
    c[2] = psi * n2 - ps * ((4.0 * s - 1.0) * inv_h) + 4.0 * m;
  } else if constexpr (DIP) {
    c[0] = psi * n0 - ps * ((4.0 * s - 3.0) * inv_h);
    c[1] = psi * n1 - ps * ((4.0 - 8.0 * s) * inv_h);
    c[2] = psi * n2 - ps * ((4.0 * s - 1.0) * inv_h);
  } else {
    c[0] = psi * n0;
    c[1] = psi * n1;
    c[2] = psi * n2;
  }
  deposit_nodes<MODE, 3>(sacc, seg, j, node, c);
}

// Second moments M = (Mqq, Mqp, Mpp) of a k = 3 particle under the two sub-flows of the
// splitting (the Lie-Poisson bracket of the quadratic phase-space polynomials gives the
// covariance equations of the linearised flow, M -> A M A^T): the kick by tau with curvature
// g (Q and Mqq frozen), A = [[1, 0], [-tau g, 1]]; the drift by tau (Mpp frozen),
// A = [[1, tau], [0, 1]].  The plain definition's operation order.
__device__ __forceinline__ void moments_kick(double tau, double g, double Mqq, double& Mqp,
                                             double& Mpp) {
  Mpp = Mpp - 2.0 * tau * g * Mqp + (tau * g) * (tau * g) * Mqq;
  Mqp = Mqp - tau * g * Mqq;
}
__device__ __forceinline__ void moments_drift(double tau, double& Mqq, double& Mqp, double Mpp) {
  Mqq = Mqq + 2.0 * tau * Mqp + tau * tau * Mpp;
  Mqp = Mqp + tau * Mpp;
}

// The prescribed potential's part of a k = 3 particle: its third derivative at Q, which adds
// -(1/2) Mqq V'''(Q) to dq*/dt (the mean force over the particle's spread), and
// (1/2) Mqq V''(Q) added to U.
__device__ __forceinline__ void k3_external(const InstDev& d, double Q, double Mqq, double& g3,
                                            double& U) {
  g3 = 0.0;
  if (!d.ext_on) return;
  const double ph = d.ext_k * Q;
  const double sn = sin(ph), cs = cos(ph);
  g3 = -(d.ext_akk * d.ext_k) * sn;
  U += 0.5 * Mqq * (d.ext_akk * cs);
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

// wave_sum of N values at once: each step of the scan is taken for all N values before the
// next, so one value's DPP latency overlaps the others'; every value gets exactly the
// additions, in the order, that wave_sum gives it.
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x111, 0xf, true>(v[i]);   // row_shr:1
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x112, 0xf, true>(v[i]);   // row_shr:2
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x114, 0xf, true>(v[i]);   // row_shr:4
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x118, 0xf, true>(v[i]);   // row_shr:8
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x142, 0xa, false>(v[i]);  // row_bcast:15
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<0x143, 0xc, false>(v[i]);  // row_bcast:31
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_bcast63(v[i]);
}

// Exclusive prefix over lanes of one value per lane.
__device__ __forceinline__ double wave_excl_scan(double v, int /*lane*/) {
  return wave_incl_scan(v) - v;
}

// Radix-2 FFT by one wavefront on (re, im) in LDS, input in bit-reversed order; tw holds
// cos/sin(2 pi k / Ng) for k < Ng/2 (LDS).
static __device__ void fft_wave(double* re, double* im, int ng, int m, const double* tw, bool inverse,
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

static __device__ void bit_reverse_wave(double* re, double* im, int ng, int m, int lane) {
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
  const double inv_ng = inv_pow2(d.log2ng);  // ng is a power of two
  const double mean = solve_total(red, 0) * inv_ng;

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
      const double C = -solve_total(red, 2) * inv_ng;
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
  // g below reads only b~, complete since the scan's barrier (the FFT path's first): this
  // barrier is for the summary totals, the FFT's E (written by one wave) and phi
  if (want_sum || use_fft || phi) __syncthreads();  // bt, E and the summary totals complete
  if (want_sum) {
    sum[0] = 0.5 * d.h * solve_total(red, 3);
    sum[1] = solve_total(red, 4) * inv_ng;
    sum[2] = solve_total(red, 5) * inv_ng;
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
      const double Pm = solve_total(red, 2) * inv_ng;
#pragma unroll
      for (int k = 0; k < kSolvePer; ++k)
        if (k < per) phi[j0 + k] = -d.h * ((P[k] + poff) - Pm);
    }
  }
  __syncthreads();
}

// Record of integer step `step` (kinetic and potential sums of that step's pass, field
// summary of its field) into slot `slot` of the history ring, which the caller keeps equal
// to step mod hist_cap; flags non-finite values.  One thread.
static __device__ void write_record_at(const InstDev& d, int slot, long long step, double K,
                                       double mom, double chg, double U, double W, double e1r,
                                       double e1i) {
  if (!d.self_on) W = e1r = e1i = 0.0;  // no field of their own acts on the particles
  VPG double* r = gp(d.hist) + (size_t)slot * kHistFields;
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
  r[11] = (double)wall_clock64();  // device constant-rate clock when the record is written
  if (!isfinite(K) || !isfinite(W) || !isfinite(U)) gp(d.scal)->nonfinite = 1;
}
// The same, the slot computed here.
static __device__ void write_record(const InstDev& d, long long step, double K, double mom,
                                    double chg, double U, double W, double e1r, double e1i) {
  write_record_at(d, (int)(step % d.hist_cap), step, K, mom, chg, U, W, e1r, e1i);
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
// k3 (an instance with second moments; GEN and P2 launches only): Mr holds the particle's
// (Mqq, Mqp, Mpp) in storage precision, updated in place.  Mr is only read when k3 holds, so
// a caller passes its local array unconditionally (a pointer chosen at run time between a
// local array and nullptr would keep the array out of registers).
// PEND: 1 or 0 when the caller knows the (uniform) pending flag at compile time, -1 to test
// `pend`.  CELL (float64 modes, P1 without general options): *cellr holds the element of Qr
// on entry (the element the previous push deposited at, from the same stored position) and
// receives the element of the drifted position; the gather then skips recomputing it.
template <int MODE, typename T, bool DIP = true, bool GEN = true, bool P2 = GEN, int PEND = -1,
          bool CELL = false>
__device__ __forceinline__ void push_particle(const InstDev& d, const double* fE, const double* fG,
                                              double* sacc, int pend, T& Qr, T& Pr, T& qsr,
                                              T& psr, const T psir, double& Ks, double& Ms,
                                              double& Cs, double& Us, bool k3in = false,
                                              T* Mr = nullptr, int* cellr = nullptr) {
  static_assert(!CELL || (!GEN && !P2 && MODE != kFP32), "CELL: float64 modes, P1, no general options");
  const bool pending = PEND < 0 ? pend != 0 : PEND == 1;
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
      if (pending) { P = P + hf * Ei; qs = qs + hf * ps * gi; }
      const double Pd = P, qd = qs, wd = psi;
      Ks += 0.5 * wd * Pd * Pd + qd * Pd;
      Ms += wd * Pd + qd;
      Cs += wd;
      P = P + hf * Ei;
      qs = qs + hf * ps * gi;
    } else {
      if (pending) P = P + hf * Ei;
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
    const double xq = CELL ? 0.0 : Q * inv_h;
    const int i = CELL ? *cellr : cell_of(xq, ng);
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
    // k = 3: the second moments move with the kicks and the drift (uniform per workgroup)
    const bool k3 = GEN && P2 && DIP && k3in;
    double Mqq = 0.0, Mqp = 0.0, Mpp = 0.0, g3 = 0.0;
    if (k3) {
      Mqq = Mr[0];
      Mqp = Mr[1];
      Mpp = Mr[2];
      k3_external(d, Q, Mqq, g3, Us);
    }
    if constexpr (DIP) {
      if (pending) {
        P = P + half * Ei;
        qs = qs + half * ps * gi;
        if (k3) {
          qs = qs - (0.5 * half) * Mqq * g3;
          moments_kick(half, gi, Mqq, Mqp, Mpp);
        }
      }
      Ks += 0.5 * psi * P * P + qs * P;
      if (k3) Ks += 0.5 * Mpp;
      Ms += psi * P + qs;
      Cs += psi;
      P = P + half * Ei;
      qs = qs + half * ps * gi;
      if (k3) {
        qs = qs - (0.5 * half) * Mqq * g3;
        moments_kick(half, gi, Mqq, Mqp, Mpp);
      }
    } else {
      if (pending) P = P + half * Ei;
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
    if constexpr (CELL) *cellr = j;
    const bool p2 = P2 && d.order == 2;
    if constexpr (DIP) {
      const double psn = ps - dt * qs;
      const T pss = (T)psn;
      const double psd = pss;
      if (k3) {
        // the drift moves the moments; the load takes the stored (rounded) Mqq
        moments_drift(dt, Mqq, Mqp, Mpp);
        const T m0 = (T)Mqq;
        Mr[0] = m0;
        Mr[1] = (T)Mqp;
        Mr[2] = (T)Mpp;
        deposit_p2<MODE, true, true>(sacc, ng, j, s, psi, psd, inv_h, (double)m0, d.seg != 0);
      } else if (p2) {
        deposit_p2<MODE, true>(sacc, ng, j, s, psi, psd, inv_h, 0.0, d.seg != 0);
      } else {
        const int node[2] = {j, (j + 1) & (ng - 1)};
        double c[2] = {psi * (1.0 - s) + psd * inv_h, psi * s - psd * inv_h};
        deposit_nodes<MODE, 2>(sacc, d.seg != 0, j, node, c);
      }
      qsr = (T)qs; psr = pss;
    } else {
      if (p2) {
        deposit_p2<MODE, false>(sacc, ng, j, s, psi, 0.0, inv_h, 0.0, d.seg != 0);
      } else {
        const int node[2] = {j, (j + 1) & (ng - 1)};
        double c[2] = {psi * (1.0 - s), psi * s};
        deposit_nodes<MODE, 2>(sacc, d.seg != 0, j, node, c);
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

}  // namespace vpk

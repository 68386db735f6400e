// HIP kernels (gfx950) for the decorated-particle cycle of arXiv 2605.21794, Section 5:
// deposit of the monopole + dipole load (eq. rhs-assembly), periodic P1 Poisson solve with
// the zero-mean gauge (eq. lin-sys), gather of E = -phi_h' and of the projected phi_h'',
// and the kick / drift sub-flows of eq. sw-evolution.
//
// Layout: particles are five structure-of-arrays streams; one workgroup owns one tile of
// consecutive particles of one instance, so every load and store is coalesced.  The
// instance's field (E, g) is staged in LDS; the load vector is accumulated into an
// LDS-private copy of the grid (float64 LDS atomics, or float32 (hi, lo) two-sum pairs
// under a 64-bit compare-and-swap, or float32 atomics in the naive mode), and each tile
// adds its grid into one of the instance's spread global accumulator copies.  In the fused
// step the last workgroup to finish an instance (ticket counter) runs that instance's
// solve in LDS, so one kernel per step advances every instance.
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
// [0, 2*Ng) doubles: field E then g (float copies for kFP32); [2*Ng, 3*Ng): accumulator
// (Ng doubles / Ng packed float (hi, lo) pairs / Ng floats).  The solve reuses [0, 4*Ng).
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
    for (int j = threadIdx.x; j < ng; j += TPB) sacc[j] = 0.0;
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

// Add the LDS grid into the global accumulator copy `copy` of the instance (device-scope
// atomics; only non-zero nodes).
template <int MODE, int TPB>
__device__ void flush(const InstDev& d, const double* sacc, int copy) {
  const int ng = d.ng;
  if constexpr (MODE == kFP32) {
    const float* a = reinterpret_cast<const float*>(sacc);
    VPG float* gacc = gp<float>(d.acc) + (size_t)copy * ng;
    for (int j = threadIdx.x; j < ng; j += TPB) {
      const float v = a[j];
      if (v != 0.0f) gadd(gacc + j, v);
    }
  } else if constexpr (MODE == kFP32TwoSum) {
    const unsigned long long* wv = reinterpret_cast<const unsigned long long*>(sacc);
    VPG double* gacc = gp(d.acc) + (size_t)copy * ng;
    for (int j = threadIdx.x; j < ng; j += TPB) {
      const unsigned long long w = wv[j];
      const double v = (double)__uint_as_float((unsigned)(w & 0xffffffffull)) +
                       (double)__uint_as_float((unsigned)(w >> 32));
      if (v != 0.0) gadd(gacc + j, v);
    }
  } else {
    VPG double* gacc = gp(d.acc) + (size_t)copy * ng;
    for (int j = threadIdx.x; j < ng; j += TPB) {
      const double v = sacc[j];
      if (v != 0.0) gadd(gacc + j, v);
    }
  }
}

// Count this workgroup's tile as done; true in the workgroup that completes the instance.
// Every wave first waits until its own device-scope atomics (load flush and kinetic sums)
// have been performed; the ticket is then taken by one thread.  The completing workgroup
// reads those sums with device-scope loads.  No cache write-back is needed because all
// cross-workgroup data of the pass travels through device-scope atomics.
__device__ bool arrive(const InstDev& d, int* sflag) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    VPG InstScal* sc = gp(d.scal);
    const unsigned prev = __hip_atomic_fetch_add(&sc->ticket, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    *sflag = (prev + 1u == (unsigned)d.ntiles) ? 1 : 0;
  }
  __syncthreads();
  return *sflag != 0;
}


// ------------------------------------------------------------------ Poisson solve
// The solve runs on ONE wavefront (64 lanes) so that it needs no workgroup barrier: lane l
// owns the contiguous nodes [l*per, (l+1)*per), per = ceil(Ng / 64), and cross-lane sums and
// scans go through shuffles.  LDS traffic between lanes stays inside the wavefront, whose
// LDS operations execute in issue order.

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

// Solve for one instance by one workgroup, LDS scratch of 4*Ng doubles at `sm` plus
// kSolveScal doubles at `ss`:
//   b_j   = sum of the accumulator copies (then cleared);
//   b~_j  = b_j - mean(b)                                  (float64, eq. neutrality);
//   E, Phi from A Phi = b~, 1^T Phi = 0                     (scan or FFT);
//   g_e   = -(b~_e + b~_{e+1}) / (2h)   (lumped projection of E onto P1, differentiated;
//           equal to -(E_{e+1} - E_{e-1}) / (2h) by (A Phi)_j = E_j - E_{j-1});
//   W     = (1/2) h sum_e E_e^2;  E1 = (1/Ng) sum_e E_e exp(-2 pi i e / Ng).
// With `record`, first write the record of the integer step whose particle pass just ran
// (kinetic sums of the pass + the field summary of the previous solve) and advance.
// Three phases: every thread loads (one memory round trip), wavefront 0 computes in LDS
// without workgroup barriers, every thread stores.  All threads of the workgroup call it.
constexpr int kSolveScal = 9;

template <int MODE, int TPB>
__device__ __forceinline__ void solve_block(const InstDev& d, double* sm, double* ss, bool record) {
  const int ng = d.ng, mask = ng - 1, halfn = ng >> 1;
  const int tid = threadIdx.x, lane = tid & 63;
  double* bt = sm;            // b, then b~
  double* tw = sm + ng;       // cos / sin (2 pi t / Ng), t < Ng/2, interleaved
  double* re = sm + 2 * ng;   // prefix sums / FFT real part, then Phi
  double* im = sm + 3 * ng;   // FFT imaginary part, then E
  double* E = im;
  const int copies = d.acc_copies;
  VPG InstScal* sc = gp(d.scal);

  // ---- phase 1: loads (and clearing of the accumulators)
  {
    const VPG double* tw_g = gp(d.tw);
    for (int j = tid; j < ng; j += TPB) {
      double t[VP_MAX_ACC_COPIES];
#pragma unroll
      for (int c = 0; c < VP_MAX_ACC_COPIES; ++c) {
        t[c] = 0.0;
        if (c < copies) {
          if constexpr (MODE == kFP32)
            t[c] = (double)gld(gp<float>(d.acc) + (size_t)c * ng + j);
          else
            t[c] = gld(gp(d.acc) + (size_t)c * ng + j);
        }
      }
      double b = 0.0;
#pragma unroll
      for (int c = 0; c < VP_MAX_ACC_COPIES; ++c) b += t[c];
      bt[j] = b;
      tw[j] = tw_g[j];
      for (int c = 0; c < copies; ++c) {
        if constexpr (MODE == kFP32)
          gst(gp<float>(d.acc) + (size_t)c * ng + j, 0.0f);
        else
          gst(gp(d.acc) + (size_t)c * ng + j, 0.0);
      }
    }
    if (record && tid == 0) {
      ss[0] = gld(&sc->K);
      ss[1] = gld(&sc->mom);
      ss[2] = gld(&sc->chg);
      ss[3] = sc->W;
      ss[4] = sc->e1r;
      ss[5] = sc->e1i;
    }
  }
  __syncthreads();

  // ---- phase 2: wavefront 0 solves (lane l owns nodes [l*per, l*per + cnt), in registers)
  if (tid < 64) {
    constexpr int kMaxPer = VP_MAX_NG / 64;
    const int per = (ng + 63) / 64;
    const int j0 = lane * per;
    const int cnt = (j0 < ng) ? min(per, ng - j0) : 0;
    const double h = d.h, inv_h = d.inv_h;
    double x[kMaxPer], Ev[kMaxPer];
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
      x[k] = (k < cnt) ? bt[j0 + k] : 0.0;
      part += x[k];
    }
    const double mean = wave_sum(part) / (double)ng;
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k)
      if (k < cnt) {
        x[k] = x[k] - mean;
        bt[j0 + k] = x[k];
      }
    if (d.solver == VP_SOLVE_FFT) {
      __builtin_amdgcn_wave_barrier();
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
#pragma unroll
      for (int k = 0; k < kMaxPer; ++k)
        if (k < cnt) {
          const int e = j0 + k;
          Ev[k] = -(re[(e + 1) & mask] - re[e]) * inv_h;
        }
    } else {
      // Gauss law: E_e = C + sum_{j=1..e} b~_j with C such that sum_e E_e = 0; then
      // Phi_e = Phi_0 - h sum_{k<e} E_k with sum_j Phi_j = 0.
      double run = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxPer; ++k)
        if (k < cnt) {
          run += (j0 + k == 0) ? 0.0 : x[k];
          Ev[k] = run;
        }
      const double off = wave_excl_scan(run, lane);
      double tp = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxPer; ++k)
        if (k < cnt) {
          Ev[k] = Ev[k] + off;
          tp += Ev[k];
        }
      const double C = -wave_sum(tp) / (double)ng;
      double run2 = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxPer; ++k)
        if (k < cnt) {
          Ev[k] = Ev[k] + C;
          x[k] = run2;  // exclusive prefix of E within the lane
          run2 += Ev[k];
        }
      const double off2 = wave_excl_scan(run2, lane);
      double up = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxPer; ++k)
        if (k < cnt) {
          x[k] = x[k] + off2;
          up += x[k];
        }
      const double Um = wave_sum(up) / (double)ng;
#pragma unroll
      for (int k = 0; k < kMaxPer; ++k)
        if (k < cnt) re[j0 + k] = -h * (x[k] - Um);  // Phi
    }
    double wpart = 0.0, e1r = 0.0, e1i = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k)
      if (k < cnt) {
        const int e = j0 + k;
        const double Ee = Ev[k];
        E[e] = Ee;
        wpart += Ee * Ee;
        const int t = e & (halfn - 1);
        const double sg = (e < halfn) ? 1.0 : -1.0;  // cos/sin of theta + pi
        e1r += Ee * (sg * tw[2 * t]);
        e1i -= Ee * (sg * tw[2 * t + 1]);
      }
    const double Wn = 0.5 * h * wave_sum(wpart);
    const double E1r = wave_sum(e1r) / (double)ng;
    const double E1i = wave_sum(e1i) / (double)ng;
    if (lane == 0) {
      ss[6] = Wn;
      ss[7] = E1r;
      ss[8] = E1i;
    }
  }
  __syncthreads();

  // ---- phase 3: stores
  {
    VPG double* bt_g = gp(d.bt);
    VPG double* E_g = gp(d.E);
    VPG double* g_g = gp(d.g);
    VPG double* Phi_g = gp(d.Phi);
    VPG float* Ef_g = gp(d.Ef);
    VPG float* gf_g = gp(d.gf);
    const double half_inv_h = 0.5 * d.inv_h;
    for (int e = tid; e < ng; e += TPB) {
      const double Ee = E[e];
      const double b0 = bt[e];
      const double g = -(b0 + bt[(e + 1) & mask]) * half_inv_h;
      bt_g[e] = b0;
      E_g[e] = Ee;
      Ef_g[e] = (float)Ee;
      g_g[e] = g;
      gf_g[e] = (float)g;
      Phi_g[e] = re[e];
    }
    if (tid == 0) {
      const double Wn = ss[6];
      if (record) {
        const long long step = sc->step;
        const double K = ss[0], mom = ss[1], chg = ss[2], Wold = ss[3];
        VPG double* r = gp(d.hist) + (size_t)(step % d.hist_cap) * kHistFields;
        r[0] = (double)step;
        r[1] = (double)step * d.dt;
        r[2] = K;
        r[3] = Wold;
        r[4] = K + Wold;
        r[5] = chg;
        r[6] = mom;
        r[7] = sqrt(2.0 * Wold / d.L);
        r[8] = ss[4];
        r[9] = ss[5];
        if (!isfinite(K) || !isfinite(Wold)) sc->nonfinite = 1;
        gst(&sc->K, 0.0);
        gst(&sc->mom, 0.0);
        gst(&sc->chg, 0.0);
        sc->step = step + 1;
        sc->pending = 1;
      }
      sc->W = Wn;
      sc->e1r = ss[7];
      sc->e1i = ss[8];
      if (!isfinite(Wn)) sc->nonfinite = 1;
      __hip_atomic_store(&sc->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
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

// One fused step for every tile: [pending half-kick] -> kinetic sums at the integer step
// -> half-kick -> drift -> deposit of the drifted state -> (last workgroup) solve.
// Thread t handles particles tile.begin + k * TPB + t, k < ppt, kGroup at a time with all
// loads of a group issued before any use; the first group is in flight while the field is
// staged in LDS.
constexpr int kGroup = 4;

template <int MODE, int TPB>
__global__ __launch_bounds__(TPB) void k_fused(const InstDev* __restrict__ insts,
                                               const Tile* __restrict__ tiles, int tile0,
                                               int ppt) {
  extern __shared__ double smem[];
  __shared__ double red[3 * (TPB / 64)];
  __shared__ double ss[kSolveScal];
  __shared__ int sflag;
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  VPG T* __restrict__ Qp = gp<T>(d.Q);
  VPG T* __restrict__ Pp = gp<T>(d.P);
  VPG T* __restrict__ qsp = gp<T>(d.qs);
  VPG T* __restrict__ psp = gp<T>(d.ps);
  const VPG T* __restrict__ psip = gp<T>(d.psi);
  double* fld = smem;
  double* sacc = smem + 2 * ng;
  double Ks = 0.0, Ms = 0.0, Cs = 0.0;
  int pend = 0;

  for (int k0 = 0; k0 < ppt; k0 += kGroup) {
    T q[kGroup], p[kGroup], a[kGroup], b[kGroup], w[kGroup];
    long long idx[kGroup];
    bool v[kGroup];
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int loc = (k0 + u) * TPB + (int)threadIdx.x;
      v[u] = (k0 + u < ppt) && (loc < tl.count);
      idx[u] = tl.begin + loc;
      if (v[u]) {
        q[u] = Qp[idx[u]]; p[u] = Pp[idx[u]]; a[u] = qsp[idx[u]]; b[u] = psp[idx[u]];
        w[u] = psip[idx[u]];
      }
    }
    if (k0 == 0) {  // the field is staged while the first group's loads are in flight
      stage<MODE, TPB>(d, fld, sacc, true, true);
      pend = gp(d.scal)->pending;
    }
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      if (!v[u]) continue;
      if constexpr (MODE == kFP32) {
        const float* fE = reinterpret_cast<const float*>(fld);
        const float* fG = fE + ng;
        float* fa = reinterpret_cast<float*>(sacc);
        const float Lf = (float)d.L, ihf = (float)d.inv_h, dtf = (float)d.dt, hf = 0.5f * dtf;
        float Q = q[u], P = p[u], qs = a[u], ps = b[u];
        const float psi = w[u];
        const int i = cell_of_f(Q * ihf, ng);
        const float Ei = fE[i], gi = fG[i];
        if (pend) { P = P + hf * Ei; qs = qs + hf * ps * gi; }
        const double Pd = P, qd = qs, wd = psi;
        Ks += 0.5 * wd * Pd * Pd + qd * Pd;
        Ms += wd * Pd + qd;
        Cs += wd;
        P = P + hf * Ei;
        qs = qs + hf * ps * gi;
        float Qn = Q + dtf * P;
        if (Qn < 0.0f) Qn += Lf;
        if (Qn >= Lf) Qn -= Lf;
        ps = ps - dtf * qs;
        Qp[idx[u]] = Qn; Pp[idx[u]] = P; qsp[idx[u]] = qs; psp[idx[u]] = ps;
        const float x = Qn * ihf;
        const int j = cell_of_f(x, ng);
        const float s = frac01_f(x, j);
        atomicAdd(fa + j, psi * (1.0f - s) + ps * ihf);
        atomicAdd(fa + ((j + 1) & (ng - 1)), psi * s - ps * ihf);
      } else {
        const double L = d.L, inv_h = d.inv_h, dt = d.dt, half = 0.5 * d.dt;
        const double Q = q[u], psi = w[u];
        double P = p[u], qs = a[u], ps = b[u];
        const int i = cell_of(Q * inv_h, ng);
        const double Ei = fld[i], gi = fld[ng + i];
        if (pend) { P = P + half * Ei; qs = qs + half * ps * gi; }
        Ks += 0.5 * psi * P * P + qs * P;
        Ms += psi * P + qs;
        Cs += psi;
        P = P + half * Ei;
        qs = qs + half * ps * gi;
        double Qn = Q + dt * P;
        if (Qn < 0.0) Qn += L;
        if (Qn >= L) Qn -= L;
        const double psn = ps - dt * qs;
        const T Qs = (T)Qn, pss = (T)psn;
        Qp[idx[u]] = Qs; Pp[idx[u]] = (T)P; qsp[idx[u]] = (T)qs; psp[idx[u]] = pss;
        const double Qd = Qs, psd = pss;
        const double x = Qd * inv_h;
        const int j = cell_of(x, ng);
        const double s = frac01(x, j);
        lds_add<MODE>(sacc, j, psi * (1.0 - s) + psd * inv_h);
        lds_add<MODE>(sacc, (j + 1) & (ng - 1), psi * s - psd * inv_h);
      }
    }
  }
  if (ppt <= 0) {  // no particle work: still stage (zero the LDS grid) before the flush
    stage<MODE, TPB>(d, fld, sacc, false, true);
  }

  // kinetic sums: wave butterflies, one barrier, one thread adds the workgroup totals
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  Ks = wave_sum(Ks);
  Ms = wave_sum(Ms);
  Cs = wave_sum(Cs);
  if (lane == 0) {
    red[3 * wid] = Ks;
    red[3 * wid + 1] = Ms;
    red[3 * wid + 2] = Cs;
  }
  __syncthreads();  // also completes every LDS deposit of the workgroup
  if (threadIdx.x == 0) {
    double kb = 0.0, mb = 0.0, cbs = 0.0;
    for (int w = 0; w < TPB / 64; ++w) {
      kb += red[3 * w];
      mb += red[3 * w + 1];
      cbs += red[3 * w + 2];
    }
    VPG InstScal* sc = gp(d.scal);
    gadd(&sc->K, kb);
    gadd(&sc->mom, mb);
    gadd(&sc->chg, cbs);
  }
  flush<MODE, TPB>(d, sacc, tl.local % d.acc_copies);
  if (arrive(d, &sflag)) solve_block<MODE, TPB>(d, smem, ss, true);
}

// Deposit of the current state only (eq. rhs-assembly), added to the global accumulator.
template <int MODE, int TPB>
__global__ __launch_bounds__(TPB) void k_deposit(const InstDev* __restrict__ insts,
                                                 const Tile* __restrict__ tiles, int tile0,
                                                 int ppt) {
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
      lds_add<MODE>(sacc, j, psi * (1.0 - s) + psd * inv_h);
      lds_add<MODE>(sacc, (j + 1) & (ng - 1), psi * s - psd * inv_h);
    }
    VP_TILE_LOOP_END
  }
  __syncthreads();
  flush<MODE, TPB>(d, sacc, tl.local % d.acc_copies);
}

// Kick by `kick` then drift by `drift` with the current field.  With use_pending, the kick of
// each instance is dt/2 when its half-kick is pending and 0 otherwise, and drift is 0.
template <int MODE, int TPB>
__global__ __launch_bounds__(TPB) void k_gather_push(const InstDev* __restrict__ insts,
                                                     const Tile* __restrict__ tiles, int tile0,
                                                     int ppt, double kick_in, double drift_in,
                                                     int use_pending) {
  extern __shared__ double smem[];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  double kick = kick_in, drift = drift_in;
  if (use_pending) {
    kick = gp(d.scal)->pending ? 0.5 * d.dt : 0.0;
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
      const int i = cell_of_f(Q * ihf, ng);
      P = P + kf * fE[i];
      qs = qs + kf * ps * fG[i];
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
      const int i = cell_of(Q * inv_h, ng);
      P = P + kick * smem[i];
      qs = qs + kick * ps * smem[ng + i];
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
                                              int ppt) {
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
  const int pend = gp(d.scal)->pending;
  double Ks = 0.0, Ms = 0.0, Cs = 0.0;
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
      if (pend) {
        const int i = cell_of_f(Q * ihf, ng);
        P = P + hf * fE[i];
        qs = qs + hf * ps * fG[i];
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
      if (pend) {
        const int i = cell_of(Q * inv_h, ng);
        P = P + half * smem[i];
        qs = qs + half * ps * smem[ng + i];
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
  if (threadIdx.x == 0) {
    VPG InstScal* sc = gp(d.scal);
    gadd(&sc->Kd, Kb);
    gadd(&sc->momd, Mb);
    gadd(&sc->chgd, Cb);
  }
}

// One workgroup per listed slot: solve and refresh the field summary (no record).
template <int MODE>
__global__ __launch_bounds__(256) void k_solve(const InstDev* __restrict__ insts,
                                               const int* __restrict__ slots) {
  extern __shared__ double smem[];
  __shared__ double ss[kSolveScal];
  const InstDev& d = insts[slots[blockIdx.x]];
  solve_block<MODE, 256>(d, smem, ss, false);
}

__global__ void k_slot_scalars(const InstDev* __restrict__ insts, const int* __restrict__ slots,
                               int nslots, int op) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  VPG InstScal* sc = gp(insts[slots[t]].scal);
  if (op == kScalClearDiag) {
    sc->Kd = 0.0; sc->momd = 0.0; sc->chgd = 0.0;
  } else if (op == kScalClearPending) {
    sc->pending = 0;
  } else {
    sc->K = sc->mom = sc->chg = 0.0;
    sc->Kd = sc->momd = sc->chgd = 0.0;
    sc->W = sc->e1r = sc->e1i = 0.0;
    sc->step = 0;
    sc->pending = 0;
    sc->ticket = 0u;
    sc->nonfinite = 0;
  }
}

__global__ void k_fill_zero(unsigned long long* p, size_t n8) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n8; i += stride) p[i] = 0ull;
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

WsLayout workspace_layout(int ng, int hist_cap) {
  WsLayout w{};
  size_t o = 0;
  w.acc = o;     o = align256(o + (size_t)VP_MAX_ACC_COPIES * ng * sizeof(double));
  w.E = o;       o = align256(o + (size_t)ng * sizeof(double));
  w.g = o;       o = align256(o + (size_t)ng * sizeof(double));
  w.Ef = o;      o = align256(o + (size_t)ng * sizeof(float));
  w.gf = o;      o = align256(o + (size_t)ng * sizeof(float));
  w.Phi = o;     o = align256(o + (size_t)ng * sizeof(double));
  w.bt = o;      o = align256(o + (size_t)ng * sizeof(double));
  w.tw = o;      o = align256(o + (size_t)ng * sizeof(double));
  w.inv_lam = o; o = align256(o + (size_t)ng * sizeof(double));
  w.scal = o;    o = align256(o + sizeof(InstScal));
  w.hist = o;    o = align256(o + (size_t)hist_cap * kHistFields * sizeof(double));
  w.total = o;
  return w;
}

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
                        int ntiles, int ppt, int max_ng, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_fused, dim3(ntiles), dim3(tpb), particle_lds_bytes(mode, max_ng), s,
              d_inst, d_tiles, tile0, ppt);
  return hipGetLastError();
}

hipError_t launch_deposit(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                          int ntiles, int ppt, int max_ng, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_deposit, dim3(ntiles), dim3(tpb), particle_lds_bytes(mode, max_ng), s,
              d_inst, d_tiles, tile0, ppt);
  return hipGetLastError();
}

hipError_t launch_gather_push(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles,
                              int tile0, int ntiles, int ppt, int max_ng, double kick, double drift,
                              hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_gather_push, dim3(ntiles), dim3(tpb),
              (size_t)2 * max_ng * sizeof(double), s, d_inst, d_tiles, tile0, ppt, kick, drift, 0);
  return hipGetLastError();
}

hipError_t launch_settle(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                         int ntiles, int ppt, int max_ng, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_gather_push, dim3(ntiles), dim3(tpb),
              (size_t)2 * max_ng * sizeof(double), s, d_inst, d_tiles, tile0, ppt, 0.0, 0.0, 1);
  return hipGetLastError();
}

hipError_t launch_diag(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                       int ntiles, int ppt, int max_ng, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_diag, dim3(ntiles), dim3(tpb), (size_t)2 * max_ng * sizeof(double), s,
              d_inst, d_tiles, tile0, ppt);
  return hipGetLastError();
}

hipError_t launch_solve(int mode, const InstDev* d_inst, const int* d_slots, int nslots,
                        int max_ng, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  const size_t lds = lds_doubles_per_node() * (size_t)max_ng * sizeof(double);
  if (mode == kFP64 || mode == kFP32TwoSum)
    hipLaunchKernelGGL(k_solve<kFP64>, dim3(nslots), dim3(256), lds, s, d_inst, d_slots);
  else if (mode == kFP32Comp)
    hipLaunchKernelGGL(k_solve<kFP32Comp>, dim3(nslots), dim3(256), lds, s, d_inst, d_slots);
  else
    hipLaunchKernelGGL(k_solve<kFP32>, dim3(nslots), dim3(256), lds, s, d_inst, d_slots);
  return hipGetLastError();
}

hipError_t launch_slot_scalars(const InstDev* d_inst, const int* d_slots, int nslots, int op,
                               hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_scalars, dim3((nslots + 63) / 64), dim3(64), 0, s, d_inst, d_slots,
                     nslots, op);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n8 = bytes / 8;
  if (n8 == 0) return hipSuccess;
  size_t blocks = (n8 + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<unsigned long long*>(p), n8);
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

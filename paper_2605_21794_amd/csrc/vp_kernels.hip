// HIP kernels (gfx950) for the decorated-particle cycle of arXiv 2605.21794, Section 5:
// deposit of the monopole + dipole load (eq. rhs-assembly), periodic P1 Poisson solve with
// the zero-mean gauge (eq. lin-sys), gather of E = -phi_h' and of the projected phi_h'',
// and the kick / drift sub-flows of eq. sw-evolution.
//
// Layout: particles are five structure-of-arrays streams; one workgroup of 256 threads
// owns one tile of consecutive particles of one instance, so every load and store is
// coalesced.  The instance's field (E, g) is staged in LDS and the load vector is
// accumulated into an LDS-private copy of the grid, which the workgroup adds into the
// instance's global accumulator once (Ng float64 atomics per tile).  The fused step's
// last workgroup of an instance (ticket counter) runs that instance's solve in LDS.
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

// Deterministic workgroup sum (fixed shuffle tree, then the four wave totals in order).
__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// ------------------------------------------------------------------ LDS staging
// Field region: 2*Ng doubles (E then g; float copies for kFP32).  Accumulator region:
// Ng*8 bytes (Ng doubles; Ng (hi, lo) float pairs for kFP32Comp; Ng floats for kFP32).
template <int MODE>
__device__ void stage(const InstDev& d, double* fld, double* sacc, bool need_field,
                      bool need_acc) {
  const int ng = d.ng;
  if (need_field) {
    if constexpr (MODE == kFP32) {
      float* f = reinterpret_cast<float*>(fld);
      for (int j = threadIdx.x; j < ng; j += kBlock) {
        f[j] = d.Ef[j];
        f[ng + j] = d.gf[j];
      }
    } else {
      for (int j = threadIdx.x; j < ng; j += kBlock) {
        fld[j] = d.E[j];
        fld[ng + j] = d.g[j];
      }
    }
  }
  if (need_acc)
    for (int j = threadIdx.x; j < ng; j += kBlock) sacc[j] = 0.0;
  __syncthreads();
}

// Add one nodal contribution c into the LDS grid.
template <int MODE>
__device__ __forceinline__ void lds_add(double* sacc, int ng, int j, double c) {
  if constexpr (MODE == kFP64) {
    atomicAdd(sacc + j, c);
  } else {
    // float (hi, lo): c is split exactly into ch + cl; ch is added with a returning atomic,
    // and the rounding error of that very addition (two-sum of the returned old value and
    // ch) is added, with cl, into lo.
    float* hi = reinterpret_cast<float*>(sacc);
    float* lo = hi + ng;
    const float ch = (float)c;
    const float cl = (float)(c - (double)ch);
    const float old = atomicAdd(hi + j, ch);
    const float s = old + ch;
    const float bp = s - old;
    const float err = (old - (s - bp)) + (ch - bp);
    atomicAdd(lo + j, err + cl);
  }
}

// Add the LDS grid into the global accumulator copy `copy` of the instance.
template <int MODE>
__device__ void flush(const InstDev& d, const double* sacc, int copy) {
  const int ng = d.ng;
  if constexpr (MODE == kFP32) {
    const float* a = reinterpret_cast<const float*>(sacc);
    float* gacc = reinterpret_cast<float*>(d.acc) + (size_t)copy * ng;
    for (int j = threadIdx.x; j < ng; j += kBlock) {
      const float v = a[j];
      if (v != 0.0f) unsafeAtomicAdd(gacc + j, v);
    }
  } else if constexpr (MODE == kFP32Comp) {
    const float* hi = reinterpret_cast<const float*>(sacc);
    const float* lo = hi + ng;
    double* gacc = d.acc + (size_t)copy * ng;
    for (int j = threadIdx.x; j < ng; j += kBlock) {
      const double v = (double)hi[j] + (double)lo[j];
      if (v != 0.0) unsafeAtomicAdd(gacc + j, v);
    }
  } else {
    double* gacc = d.acc + (size_t)copy * ng;
    for (int j = threadIdx.x; j < ng; j += kBlock) {
      const double v = sacc[j];
      if (v != 0.0) unsafeAtomicAdd(gacc + j, v);
    }
  }
}

// Count this workgroup's tile as done; true in the workgroup that completes the instance.
__device__ bool arrive(const InstDev& d, int* sflag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(&d.scal->ticket, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    *sflag = (prev + 1u == (unsigned)d.ntiles) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *sflag != 0;
  if (last) __threadfence();
  return last;
}

// ------------------------------------------------------------------ Poisson solve
// Radix-2 FFT on (re, im) held in bit-reversed order; tw holds cos/sin of 2 pi k / Ng.
__device__ void fft_lds(double* re, double* im, int ng, int m, const double* tw, bool inverse) {
  for (int s = 1; s <= m; ++s) {
    const int half = 1 << (s - 1);
    const int tstride = ng >> s;
    for (int b = threadIdx.x; b < (ng >> 1); b += kBlock) {
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
    __syncthreads();
  }
}

__device__ void bit_reverse_lds(double* re, double* im, int ng, int m) {
  for (int j = threadIdx.x; j < ng; j += kBlock) {
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
  __syncthreads();
}

// Solve for one instance with one workgroup: gather and clear the global load, subtract its
// mean (float64), Phi = A^+ b~ by FFT, E, g, W and the mode-1 amplitude.  With `record`,
// first write the diagnostic record of the step that just ran its particle pass (kinetic
// sums of this pass + the field summary from the previous solve) and advance the counter.
template <int MODE>
__device__ void solve_instance(const InstDev& d, double* re, double* im, double* red,
                               bool record) {
  const int ng = d.ng, m = d.log2ng, mask = ng - 1;
  const int tid = threadIdx.x;

  for (int j = tid; j < ng; j += kBlock) {
    double b = 0.0;
    for (int c = 0; c < d.acc_copies; ++c) {
      if constexpr (MODE == kFP32) {
        float* a = reinterpret_cast<float*>(d.acc) + (size_t)c * ng + j;
        b += (double)__hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a, 0.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        double* a = d.acc + (size_t)c * ng + j;
        b += __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    re[j] = b;
  }
  __syncthreads();
  double part = 0.0;
  for (int j = tid; j < ng; j += kBlock) part += re[j];
  const double mean = block_sum(part, red) / (double)ng;
  for (int j = tid; j < ng; j += kBlock) {
    const double bt = re[j] - mean;
    re[j] = bt;
    im[j] = 0.0;
    d.bt[j] = bt;
  }
  __syncthreads();

  bit_reverse_lds(re, im, ng, m);
  fft_lds(re, im, ng, m, d.tw, false);
  for (int k = tid; k < ng; k += kBlock) {
    const double il = d.inv_lam[k];
    re[k] = re[k] * il;
    im[k] = im[k] * il;
  }
  __syncthreads();
  bit_reverse_lds(re, im, ng, m);
  fft_lds(re, im, ng, m, d.tw, true);
  const double inv_ng = 1.0 / (double)ng;
  for (int j = tid; j < ng; j += kBlock) {
    const double phi = re[j] * inv_ng;
    re[j] = phi;
    d.Phi[j] = phi;
  }
  __syncthreads();
  const double inv_h = d.inv_h;
  for (int e = tid; e < ng; e += kBlock) {
    const double E = -(re[(e + 1) & mask] - re[e]) * inv_h;
    im[e] = E;
    d.E[e] = E;
    d.Ef[e] = (float)E;
  }
  __syncthreads();
  double wpart = 0.0, e1r = 0.0, e1i = 0.0;
  const int halfn = ng >> 1;
  for (int e = tid; e < ng; e += kBlock) {
    const double Em = im[(e - 1) & mask], E0 = im[e], Ep = im[(e + 1) & mask];
    const double En_a = 0.5 * (Em + E0);
    const double En_b = 0.5 * (E0 + Ep);
    const double g = -(En_b - En_a) * inv_h;
    d.g[e] = g;
    d.gf[e] = (float)g;
    wpart += E0 * E0;
    const int k = e & (halfn - 1);
    const double sg = (e < halfn) ? 1.0 : -1.0;  // cos/sin of theta + pi flip sign
    e1r += E0 * (sg * d.tw[2 * k]);
    e1i -= E0 * (sg * d.tw[2 * k + 1]);
  }
  const double Wsum = block_sum(wpart, red);
  const double E1r = block_sum(e1r, red) * inv_ng;
  const double E1i = block_sum(e1i, red) * inv_ng;
  const double Wn = 0.5 * d.h * Wsum;

  if (tid == 0) {
    InstScal* sc = d.scal;
    if (record) {
      const long long st = sc->step;
      double* r = d.hist + (size_t)(st % d.hist_cap) * kHistFields;
      const double K = __hip_atomic_load(&sc->K, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double mom = __hip_atomic_load(&sc->mom, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double chg = __hip_atomic_load(&sc->chg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double W = sc->W;
      r[0] = (double)st;
      r[1] = (double)st * d.dt;
      r[2] = K;
      r[3] = W;
      r[4] = K + W;
      r[5] = chg;
      r[6] = mom;
      r[7] = sqrt(2.0 * W / d.L);
      r[8] = sc->e1r;
      r[9] = sc->e1i;
      if (!isfinite(K) || !isfinite(W)) sc->nonfinite = 1;
      __hip_atomic_store(&sc->K, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&sc->mom, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&sc->chg, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sc->step = st + 1;
      sc->pending = 1;
    }
    sc->W = Wn;
    sc->e1r = E1r;
    sc->e1i = E1i;
    if (!isfinite(Wn)) sc->nonfinite = 1;
    __hip_atomic_store(&sc->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------------ particle passes
// Loop shape shared by the particle kernels: thread t of the workgroup handles particles
// tile.begin + k * 256 + t for k < ppt, four at a time with all loads issued first.
#define VP_TILE_LOOP_BEGIN                                                        \
  for (int k0 = 0; k0 < ppt; k0 += 4) {                                           \
    bool v[4];                                                                    \
    long long idx[4];                                                             \
    _Pragma("unroll") for (int u = 0; u < 4; ++u) {                              \
      const int loc = (k0 + u) * kBlock + (int)threadIdx.x;                       \
      v[u] = (k0 + u < ppt) && (loc < tl.count);                                  \
      idx[u] = tl.begin + loc;                                                    \
    }

#define VP_TILE_LOOP_END }

// One fused step for every tile: [pending half-kick] -> kinetic sums at the integer step
// -> half-kick -> drift -> deposit of the drifted state -> (last workgroup) solve.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_fused(const InstDev* __restrict__ insts,
                                                  const Tile* __restrict__ tiles, int tile0,
                                                  int ppt) {
  extern __shared__ double smem[];
  __shared__ double red[4];
  __shared__ int sflag;
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  double* fld = smem;
  double* sacc = smem + 2 * ng;
  stage<MODE>(d, fld, sacc, true, true);
  const int pend = d.scal->pending;
  T* __restrict__ Qp = static_cast<T*>(d.Q);
  T* __restrict__ Pp = static_cast<T*>(d.P);
  T* __restrict__ qsp = static_cast<T*>(d.qs);
  T* __restrict__ psp = static_cast<T*>(d.ps);
  const T* __restrict__ psip = static_cast<const T*>(d.psi);
  double Ks = 0.0, Ms = 0.0, Cs = 0.0;

  if constexpr (MODE == kFP32) {
    const float* fE = reinterpret_cast<const float*>(fld);
    const float* fG = fE + ng;
    const float Lf = (float)d.L, ihf = (float)d.inv_h, dtf = (float)d.dt, hf = 0.5f * dtf;
    VP_TILE_LOOP_BEGIN
    float q[4], p[4], a[4], b[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) {
        q[u] = Qp[idx[u]]; p[u] = Pp[idx[u]]; a[u] = qsp[idx[u]]; b[u] = psp[idx[u]];
        w[u] = psip[idx[u]];
      }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
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
      float* fa = reinterpret_cast<float*>(sacc);
      atomicAdd(fa + j, psi * (1.0f - s) + ps * ihf);
      atomicAdd(fa + ((j + 1) & (ng - 1)), psi * s - ps * ihf);
    }
    VP_TILE_LOOP_END
  } else {
    const double L = d.L, inv_h = d.inv_h, dt = d.dt, half = 0.5 * d.dt;
    VP_TILE_LOOP_BEGIN
    T q[4], p[4], a[4], b[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) {
        q[u] = Qp[idx[u]]; p[u] = Pp[idx[u]]; a[u] = qsp[idx[u]]; b[u] = psp[idx[u]];
        w[u] = psip[idx[u]];
      }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
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
      lds_add<MODE>(sacc, ng, j, psi * (1.0 - s) + psd * inv_h);
      lds_add<MODE>(sacc, ng, (j + 1) & (ng - 1), psi * s - psd * inv_h);
    }
    VP_TILE_LOOP_END
  }

  const double Kb = block_sum(Ks, red);
  const double Mb = block_sum(Ms, red);
  const double Cb = block_sum(Cs, red);
  if (threadIdx.x == 0) {
    unsafeAtomicAdd(&d.scal->K, Kb);
    unsafeAtomicAdd(&d.scal->mom, Mb);
    unsafeAtomicAdd(&d.scal->chg, Cb);
  }
  __syncthreads();
  flush<MODE>(d, sacc, tl.local % d.acc_copies);
  if (arrive(d, &sflag)) solve_instance<MODE>(d, fld, fld + ng, red, true);
}

// Deposit of the current state only (eq. rhs-assembly), added to the global accumulator.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_deposit(const InstDev* __restrict__ insts,
                                                    const Tile* __restrict__ tiles, int tile0,
                                                    int ppt) {
  extern __shared__ double smem[];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  double* sacc = smem + 2 * ng;
  stage<MODE>(d, smem, sacc, false, true);
  const T* __restrict__ Qp = static_cast<const T*>(d.Q);
  const T* __restrict__ psp = static_cast<const T*>(d.ps);
  const T* __restrict__ psip = static_cast<const T*>(d.psi);
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
      lds_add<MODE>(sacc, ng, j, psi * (1.0 - s) + psd * inv_h);
      lds_add<MODE>(sacc, ng, (j + 1) & (ng - 1), psi * s - psd * inv_h);
    }
    VP_TILE_LOOP_END
  }
  __syncthreads();
  flush<MODE>(d, sacc, tl.local % d.acc_copies);
}

// Kick by `kick` then drift by `drift` with the current field.  With use_pending, the kick of
// each instance is dt/2 when its half-kick is pending and 0 otherwise, and drift is 0.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_gather_push(const InstDev* __restrict__ insts,
                                                        const Tile* __restrict__ tiles,
                                                        int tile0, int ppt, double kick_in,
                                                        double drift_in, int use_pending) {
  extern __shared__ double smem[];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  double kick = kick_in, drift = drift_in;
  if (use_pending) {
    kick = d.scal->pending ? 0.5 * d.dt : 0.0;
    drift = 0.0;
  }
  if (kick == 0.0 && drift == 0.0) return;  // uniform per workgroup: no barrier skipped
  stage<MODE>(d, smem, nullptr, true, false);
  T* __restrict__ Qp = static_cast<T*>(d.Q);
  T* __restrict__ Pp = static_cast<T*>(d.P);
  T* __restrict__ qsp = static_cast<T*>(d.qs);
  T* __restrict__ psp = static_cast<T*>(d.ps);
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
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_diag(const InstDev* __restrict__ insts,
                                                 const Tile* __restrict__ tiles, int tile0,
                                                 int ppt) {
  extern __shared__ double smem[];
  __shared__ double red[4];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  stage<MODE>(d, smem, nullptr, true, false);
  const T* __restrict__ Qp = static_cast<const T*>(d.Q);
  const T* __restrict__ Pp = static_cast<const T*>(d.P);
  const T* __restrict__ qsp = static_cast<const T*>(d.qs);
  const T* __restrict__ psp = static_cast<const T*>(d.ps);
  const T* __restrict__ psip = static_cast<const T*>(d.psi);
  const int pend = d.scal->pending;
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
  const double Kb = block_sum(Ks, red);
  const double Mb = block_sum(Ms, red);
  const double Cb = block_sum(Cs, red);
  if (threadIdx.x == 0) {
    unsafeAtomicAdd(&d.scal->Kd, Kb);
    unsafeAtomicAdd(&d.scal->momd, Mb);
    unsafeAtomicAdd(&d.scal->chgd, Cb);
  }
}

// One workgroup per listed slot: solve and refresh the field summary (no record).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_solve(const InstDev* __restrict__ insts,
                                                  const int* __restrict__ slots) {
  extern __shared__ double smem[];
  __shared__ double red[4];
  const InstDev& d = insts[slots[blockIdx.x]];
  __threadfence();
  solve_instance<MODE>(d, smem, smem + d.ng, red, false);
}

__global__ void k_slot_scalars(const InstDev* __restrict__ insts, const int* __restrict__ slots,
                               int nslots, int op) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  InstScal* sc = insts[slots[t]].scal;
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
  const T* Qp = static_cast<const T*>(d.Q);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    cells[k] = cell_of((double)Qp[k] * d.inv_h, d.ng);
}

// ------------------------------------------------------------------ chunked stable sort
// Workgroup b sorts particles [b*chunk, min(n, (b+1)*chunk)) by cell (float64 index
// formula) with two stable 5-bit counting passes in LDS, then permutes the five arrays
// in place through an LDS staging buffer.
template <typename T>
__device__ void permute_array(T* __restrict__ X, long long c0, int m, const unsigned short* order,
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
  const T* Qp = static_cast<const T*>(d.Q);
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
  permute_array<T>(static_cast<T*>(d.Q), c0, m, iA, stagebuf);
  permute_array<T>(static_cast<T*>(d.P), c0, m, iA, stagebuf);
  permute_array<T>(static_cast<T*>(d.qs), c0, m, iA, stagebuf);
  permute_array<T>(static_cast<T*>(d.ps), c0, m, iA, stagebuf);
  permute_array<T>(static_cast<T*>(d.psi), c0, m, iA, stagebuf);
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

size_t particle_lds_bytes(int /*mode*/, int max_ng) { return (size_t)3 * max_ng * sizeof(double); }

#define VP_DISPATCH(mode, KERNEL, ...)                                                     \
  do {                                                                                     \
    if ((mode) == kFP64) hipLaunchKernelGGL(KERNEL<kFP64>, __VA_ARGS__);                   \
    else if ((mode) == kFP32Comp) hipLaunchKernelGGL(KERNEL<kFP32Comp>, __VA_ARGS__);      \
    else hipLaunchKernelGGL(KERNEL<kFP32>, __VA_ARGS__);                                   \
  } while (0)

hipError_t launch_fused(int mode, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                        int ntiles, int ppt, int max_ng, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, k_fused, dim3(ntiles), dim3(kBlock), particle_lds_bytes(mode, max_ng), s,
              d_inst, d_tiles, tile0, ppt);
  return hipGetLastError();
}

hipError_t launch_deposit(int mode, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                          int ntiles, int ppt, int max_ng, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, k_deposit, dim3(ntiles), dim3(kBlock), particle_lds_bytes(mode, max_ng), s,
              d_inst, d_tiles, tile0, ppt);
  return hipGetLastError();
}

hipError_t launch_gather_push(int mode, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                              int ntiles, int ppt, int max_ng, double kick, double drift,
                              hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, k_gather_push, dim3(ntiles), dim3(kBlock),
              (size_t)2 * max_ng * sizeof(double), s, d_inst, d_tiles, tile0, ppt, kick, drift, 0);
  return hipGetLastError();
}

hipError_t launch_settle(int mode, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                         int ntiles, int ppt, int max_ng, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, k_gather_push, dim3(ntiles), dim3(kBlock),
              (size_t)2 * max_ng * sizeof(double), s, d_inst, d_tiles, tile0, ppt, 0.0, 0.0, 1);
  return hipGetLastError();
}

hipError_t launch_diag(int mode, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                       int ntiles, int ppt, int max_ng, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, k_diag, dim3(ntiles), dim3(kBlock), (size_t)2 * max_ng * sizeof(double), s,
              d_inst, d_tiles, tile0, ppt);
  return hipGetLastError();
}

hipError_t launch_solve(int mode, const InstDev* d_inst, const int* d_slots, int nslots,
                        int max_ng, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  VP_DISPATCH(mode, k_solve, dim3(nslots), dim3(kBlock), (size_t)2 * max_ng * sizeof(double), s,
              d_inst, d_slots);
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

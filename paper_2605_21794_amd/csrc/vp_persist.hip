// The persistent form of the fused step (k_persist): many steps in one cooperative launch,
// the particles of each tile held in registers, with its launch and capacity query.
#include "vp_device.h"

namespace vpk {

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
  VPG unsigned* arrive = sc->arrive;
  // The tiles of the instance that count on arrival group g (lane g of the first wave waits
  // for them): local indices congruent to g mod kArriveGroups.
  const int my_group = tl.local & (kArriveGroups - 1);
  const unsigned group_tiles =
      threadIdx.x < kArriveGroups
          ? (unsigned)((d.ntiles - (int)threadIdx.x + kArriveGroups - 1) / kArriveGroups)
          : 0u;

  int r0 = phase0;
  for (int st = 0; st < nsteps; ++st) {
    // nothing is hoisted out of the step loop: keeps the step's registers per step
    __asm__ __volatile__("" ::: "memory");
    const int r1 = ring_next(r0), r2 = ring_prev(r0);
    if (st > 0) {  // wait for every tile of the instance to finish the previous step
      if (threadIdx.x < kArriveGroups) {  // one lane per arrival group, all groups at once
        const unsigned target = (unsigned)st * group_tiles;
        VPG unsigned* c = arrive + threadIdx.x * kArriveStride;
        unsigned it = 0;
        while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
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
        __hip_atomic_fetch_add(arrive + my_group * kArriveStride, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
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

}  // namespace vpk

// ckpp_plan_dev.h -- the plan's persistent lookup kernel (lookup_plan) and
// its launchers, shared by the translation units that instantiate it
// without timers (ckpp_plan.hip) and with timers (ckpp_plan_timed.hip).
#pragma once

#include "ckpp_lookup_dev.h"

namespace ckpp {

// Arguments of a plan launch.
struct PlanArgs {
  const PlanItem *items;
  uint32_t nitems;
  const uint4 *keys;
  uint8_t *found;
  uint64_t *vals;
  uint32_t *ctr;  // dynamic schedule: next item, finished waves
  TimerArgs tm;   // the time of the launch, for items on tables with timers
};

// Launches the plan kernel whose passes check times (some items are on
// tables with timers).
hipError_t launch_plan_timed(const PlanArgs &A, bool two_buffers, const ckpp_plan_launch_t &L,
                             int num_cus, hipStream_t s);

namespace {

// The wave's next work item: lane 0 takes a ticket from the plan's counter
// and the wave shares it.
__device__ __forceinline__ uint32_t take_item(uint32_t *ctr, uint32_t lane) {
  uint32_t v = 0u;
  if (lane == 0u) v = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// The item after `prev` for this wave: the wave's own stride through the
// list (static schedule) or the next ticket (dynamic schedule); once past
// the end, it stays there.
template <bool DYN>
__device__ __forceinline__ uint32_t next_item(uint32_t prev, uint32_t stride, uint32_t nitems,
                                              uint32_t *ctr, uint32_t lane) {
  if (prev >= nitems) return prev;
  return DYN ? take_item(ctr, lane) : prev + stride;
}

// Keys of one pass of an item: lookups off + 64 j + lane.
template <uint32_t PER>
__device__ __forceinline__ void item_keys(const uint4 *keys, const PlanItem &I, uint32_t off,
                                          uint32_t lane, uint4 (&k)[PER]) {
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    const uint32_t o = off + 64u * j + lane;
    k[j] = o < I.count ? load_stream(keys + I.start + o) : zero4();
  }
}

// A plan's batches in one persistent launch.  Each wave runs work items (a
// range of one table's batch, in passes of PER * 64 lookups) in a
// three-deep pipeline: while item `cur` runs, the descriptor of the next
// item is already loaded and the index of the one after is known; the last
// pass of `cur` loads the next item's first keys, the descriptor after it
// and the next index, all independent loads issued while that pass's lines
// are in flight.  DYN: items are handed out by a device counter (the wave
// that finishes last rewinds it, so the next launch or graph replay starts
// from zero without a memory set); else wave w runs items w, w + W, ...
// The passes are those of the one-table kernels.  TIMED: some
// items are on tables with timers, and every item runs the timed passes:
// at the launch's time on those, at kNoTime (no time check) on the others.
template <uint32_t WAVES, uint32_t NB, uint32_t PER, bool DYN, uint32_t LANES, bool TIMED>
__global__ void __launch_bounds__(64 * WAVES)
    lookup_plan(const PlanItem *__restrict__ items, uint32_t nitems, const uint4 *__restrict__ keys,
                uint8_t *__restrict__ found, uint64_t *__restrict__ vals, uint32_t *__restrict__ ctr,
                TimerArgs tm) {
  static_assert(LANES == 1 || PER <= 2, "8 or 4 lanes per line: one or two lookups per lane");
  constexpr uint32_t P = 64u * PER;  // lookups per pass
  __shared__ uint4 s_lines[LANES == 8 ? WAVES * NB * kWaveQuarters : 1];
  Wave w;
  if constexpr (LANES == 8) w = wave_lines<NB>(s_lines);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t stride = gridDim.x * WAVES;
  const uint32_t wave_id =
      (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * WAVES + (threadIdx.x >> 6)));
  uint32_t cur = DYN ? take_item(ctr, lane) : wave_id;
  uint32_t n1 = next_item<DYN>(cur, stride, nitems, ctr, lane);
  uint32_t n2 = next_item<DYN>(n1, stride, nitems, ctr, lane);
  const PlanItem none{nullptr, 0ull, 0ull, 0u, 0u, 0u, 0u};
  PlanItem I = cur < nitems ? items[cur] : none;
  PlanItem I1 = n1 < nitems ? items[n1] : none;
  uint4 k[PER];
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) k[j] = zero4();
  if (cur < nitems) item_keys<PER>(keys, I, 0u, lane, k);
  while (cur < nitems) {
    const uint32_t mode = I.mode & kPlanModeMask;
    TableRef T{I.tab, I.seed, I.log2b};
    if (TIMED) {
      // the timed passes serve both kinds of table: one without timers
      // runs at kNoTime and refreshes nothing
      const bool timed = (I.mode & kPlanItemTimed) != 0u;
      T.now = timed ? tm.now : kNoTime;
      T.refresh = timed ? tm.refresh : 0u;
      T.expiry = tm.expiry;
    }
    PlanItem I2 = none;
    uint32_t n3 = n2;
    for (uint32_t off = 0u; off < I.count; off += P) {
      const bool last = off + P >= I.count;
      uint4 kn[PER];
#pragma unroll
      for (uint32_t j = 0; j < PER; ++j) kn[j] = zero4();
      auto pre = [&] {
        if (!last) {
          item_keys<PER>(keys, I, off + P, lane, kn);
        } else {
          if (n1 < nitems) item_keys<PER>(keys, I1, 0u, lane, kn);
          if (n2 < nitems) I2 = items[n2];
          n3 = next_item<DYN>(n2, stride, nitems, ctr, lane);
        }
      };
      const uint64_t ia = I.start + off + lane;
      bool ok[PER];
#pragma unroll
      for (uint32_t j = 0; j < PER; ++j) ok[j] = off + 64u * j + lane < I.count;
      // the passes of the one-table kernels; NB = 2 compiles in the
      // pessimistic mode (for 8 lanes with the wave's second line buffer);
      // with NB = 1 the host passes no pessimistic item
      if constexpr (LANES == 1) {
        if (mode == kModeCuckoopp)
          reg_pass<kModeCuckoopp, TIMED, PER>(T, k, ok, found + ia, vals + ia, pre);
        else if (mode == kModeOptimistic)
          reg_pass<kModeOptimistic, TIMED, PER>(T, k, ok, found + ia, vals + ia, pre);
        else
          reg_pass<kModeBoth, TIMED, PER>(T, k, ok, found + ia, vals + ia, pre);
      } else if constexpr (LANES == 4) {
        if (mode == kModeCuckoopp)
          quad_pass<kModeCuckoopp, TIMED, PER>(T, k, ok, found + ia, vals + ia, pre);
        else if (mode == kModeOptimistic)
          quad_pass<kModeOptimistic, TIMED, PER>(T, k, ok, found + ia, vals + ia, pre);
        else if (NB == 2)
          quad_pass<kModeBoth, TIMED, PER>(T, k, ok, found + ia, vals + ia, pre);
      } else if constexpr (PER == 1) {
        if (mode == kModeCuckoopp)
          lds_pass<kModeCuckoopp, TIMED>(w, T, k[0], ok[0], found + ia, vals + ia, pre);
        else if (mode == kModeOptimistic)
          lds_pass<kModeOptimistic, TIMED>(w, T, k[0], ok[0], found + ia, vals + ia, pre);
        else if (NB == 2)
          lds_pass<kModeBoth, TIMED>(w, T, k[0], ok[0], found + ia, vals + ia, pre);
      } else {
        const uint64_t ib = ia + 64u;
        if (mode == kModeCuckoopp) {
          dual_pass<kModeCuckoopp, TIMED>(w, T, k[0], ok[0], k[1], ok[1], found + ia, vals + ia,
                                          found + ib, vals + ib, pre);
        } else if (mode == kModeOptimistic) {
          dual_pass<kModeOptimistic, TIMED>(w, T, k[0], ok[0], k[1], ok[1], found + ia,
                                            vals + ia, found + ib, vals + ib, pre);
        } else if (NB == 2) {
          lds_pass<kModeBoth, TIMED>(w, T, k[0], ok[0], found + ia, vals + ia, [] {});
          lds_pass<kModeBoth, TIMED>(w, T, k[1], ok[1], found + ib, vals + ib, pre);
        }
      }
#pragma unroll
      for (uint32_t j = 0; j < PER; ++j) k[j] = kn[j];
    }
    cur = n1;
    I = I1;
    n1 = n2;
    I1 = I2;
    n2 = n3;
  }
  if (DYN && lane == 0u) {
    // every ticket this wave will ever take is taken (each ticket's value
    // was used, so its atomic was performed): count the wave out; the last
    // one rewinds both.  Relaxed: the counters are the only words that need
    // ordering, and an acquire-release here would write back and invalidate
    // the XCD's L2 cache once per wave
    const uint32_t out = __hip_atomic_fetch_add(ctr + 1, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (out == gridDim.x * WAVES - 1u) {
      __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ctr + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <uint32_t WAVES, uint32_t NB, uint32_t PER, uint32_t LANES, bool TIMED>
hipError_t launch_plan_shape(const PlanArgs &A, const ckpp_plan_launch_t &L, int num_cus,
                             hipStream_t s) {
  // persistent grid: blocks_per_cu per CU, but no more waves than items
  const uint64_t grid = capped_grid(A.nitems, WAVES, L.blocks_per_cu, num_cus);
  if (L.schedule == CKPP_PLAN_DYNAMIC)
    hipLaunchKernelGGL((lookup_plan<WAVES, NB, PER, true, LANES, TIMED>), dim3((uint32_t)grid),
                       dim3(64 * WAVES), 0, s, A.items, A.nitems, A.keys, A.found, A.vals, A.ctr,
                       A.tm);
  else
    hipLaunchKernelGGL((lookup_plan<WAVES, NB, PER, false, LANES, TIMED>), dim3((uint32_t)grid),
                       dim3(64 * WAVES), 0, s, A.items, A.nitems, A.keys, A.found, A.vals, A.ctr,
                       A.tm);
  return hipGetLastError();
}

// The form, lookups per lane and line buffers of the launch shape.
template <uint32_t WAVES, bool TIMED>
hipError_t launch_plan_form(const PlanArgs &A, bool two, const ckpp_plan_launch_t &L,
                            int num_cus, hipStream_t s) {
  const uint32_t per = L.lookups_per_lane;
  if (L.lanes_per_lookup == 1) {
    if (per == 4) return launch_plan_shape<WAVES, 1, 4, 1, TIMED>(A, L, num_cus, s);
    if (per == 2) return launch_plan_shape<WAVES, 1, 2, 1, TIMED>(A, L, num_cus, s);
    return launch_plan_shape<WAVES, 1, 1, 1, TIMED>(A, L, num_cus, s);
  }
  if (L.lanes_per_lookup == 4) {
    if (per == 2)
      return two ? launch_plan_shape<WAVES, 2, 2, 4, TIMED>(A, L, num_cus, s)
                 : launch_plan_shape<WAVES, 1, 2, 4, TIMED>(A, L, num_cus, s);
    return two ? launch_plan_shape<WAVES, 2, 1, 4, TIMED>(A, L, num_cus, s)
               : launch_plan_shape<WAVES, 1, 1, 4, TIMED>(A, L, num_cus, s);
  }
  if (per == 2)
    return two ? launch_plan_shape<WAVES, 2, 2, 8, TIMED>(A, L, num_cus, s)
               : launch_plan_shape<WAVES, 1, 2, 8, TIMED>(A, L, num_cus, s);
  return two ? launch_plan_shape<WAVES, 2, 1, 8, TIMED>(A, L, num_cus, s)
             : launch_plan_shape<WAVES, 1, 1, 8, TIMED>(A, L, num_cus, s);
}

template <bool TIMED>
hipError_t launch_plan_block(const PlanArgs &A, bool two, const ckpp_plan_launch_t &L,
                             int num_cus, hipStream_t s) {
  switch (L.block) {
    case 64: return launch_plan_form<1, TIMED>(A, two, L, num_cus, s);
    case 128: return launch_plan_form<2, TIMED>(A, two, L, num_cus, s);
    default: return launch_plan_form<4, TIMED>(A, two, L, num_cus, s);
  }
}

}  // namespace
}  // namespace ckpp

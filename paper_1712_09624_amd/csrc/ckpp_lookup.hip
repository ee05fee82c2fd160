// ckpp_lookup.hip -- batched lookup kernel (gfx950).
//
// One lookup (Sec. 2 lookup procedure, Sec. 4.1 pruning):
//   hash the key -> primary bucket p, alternate a, tag, two bloom bits;
//   read p; a slot holds the key iff it is busy and its full 16-byte key
//   equals the searched key (its tag is only a hint that selects which keys
//   to compare); if not found, Cuckoo++ reads a only when both bloom bits
//   are set in p's filter, the pessimistic mode reads a together with p, the
//   optimistic mode reads a whenever the key was not in p;
//   write found (u8) and the value (u64, 0 on a miss).
//
// GPU form.  On MI355X every random read that misses the L2 costs one
// 128-byte line request, a later second access to the same line costs
// another, and the request rate -- not the byte rate -- bounds random reads.
// So a bucket line is read exactly once, in one instruction, by 8 lanes (16
// bytes each), straight into LDS (global_load_lds_dwordx4: the data in
// flight occupies no registers, so a wave keeps 64 line requests in flight
// at once).  Each lane owns one lookup: it hashes its key once, hands its
// bucket index to the fetching group (ds_bpermute), and after the lines
// have landed it analyses its own line from LDS: tags and busy mask, then
// the full keys of the candidate slots and the value.  The first line of a
// bucket holds the metadata and slots 0..3, so most lookups need one
// request; the second line (slots 4..7) and the secondary bucket are
// fetched, in the same cooperative way, only for the lookups of the wave
// that need them, and skipped when none does.  Keys for the next tile are
// loaded while the current tile is processed; keys stream in and results
// stream out with non-temporal accesses.
//
// Other forms of the same lookup: two lookups per lane (lookup_dual: the
// second half's lines land in registers and are parked in LDS), four lanes
// per lookup with each line spread over a quad's registers and analysed
// there (lookup_quad), one lane per lookup with bucket heads in registers
// (lookup_reg), and a plan's persistent kernel over many tables' batches
// (lookup_plan).  On a table
// with timers (Sec. 4.2) a key match counts only if the entry is alive,
// and a refreshing lookup writes the new time into the entry's value word.

#include "ckpp_lookup_dev.h"

namespace ckpp {
namespace {

// One table's batch, one lookup per lane per pass; the grid strides over
// the batch and each wave loads its next keys while its lines are in flight.
template <uint32_t WAVES, uint32_t MODE, bool TIMED>
__global__ void __launch_bounds__(64 * WAVES)
    lookup_lds(TableRef T, const uint4 *__restrict__ keys, uint64_t n,
               uint8_t *__restrict__ found, uint64_t *__restrict__ vals) {
  constexpr uint32_t NB = MODE == kModeBoth ? 2 : 1;  // line buffers per wave
  __shared__ uint4 s_lines[WAVES * NB * kWaveQuarters];
  const Wave w = wave_lines<NB>(s_lines);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint4 key = i < n ? load_stream(keys + i) : zero4();
  // the wave stays together: its loop condition is the wave's first lookup
  for (; i - w.lane < n; i += stride) {
    uint4 knext;
    lds_pass<MODE, TIMED>(w, T, key, i < n, found + i, vals + i, [&] {
      const uint64_t inext = i + stride;
      knext = inext < n ? load_stream(keys + inext) : zero4();
    });
    key = knext;
  }
}

// One table's batch, two lookups per lane per pass (lookups w0 + lane and
// w0 + 64 + lane of the wave's 128-lookup tile).
template <uint32_t WAVES, uint32_t MODE, bool TIMED>
__global__ void __launch_bounds__(64 * WAVES)
    lookup_dual(TableRef T, const uint4 *__restrict__ keys, uint64_t n,
                uint8_t *__restrict__ found, uint64_t *__restrict__ vals) {
  __shared__ uint4 s_lines[WAVES * kWaveQuarters];
  const Wave w = wave_lines<1>(s_lines);
  const uint32_t lane = w.lane;
  const uint64_t wave0 = ((uint64_t)blockIdx.x * WAVES + (threadIdx.x >> 6)) * 128u;
  const uint64_t stride = (uint64_t)gridDim.x * WAVES * 128u;
  uint4 ka = wave0 + lane < n ? load_stream(keys + wave0 + lane) : zero4();
  uint4 kb = wave0 + 64u + lane < n ? load_stream(keys + wave0 + 64u + lane) : zero4();
  for (uint64_t w0 = wave0; w0 < n; w0 += stride) {
    const uint64_t ia = w0 + lane, ib = w0 + 64u + lane;
    uint4 na, nb;
    dual_pass<MODE, TIMED>(w, T, ka, ia < n, kb, ib < n, found + ia, vals + ia, found + ib,
                           vals + ib,
                    [&] {
                      const uint64_t nx = w0 + stride;
                      na = nx + lane < n ? load_stream(keys + nx + lane) : zero4();
                      nb = nx + 64u + lane < n ? load_stream(keys + nx + 64u + lane) : zero4();
                    });
    ka = na;
    kb = nb;
  }
}

// One table's batch, four lanes per line with the lines in registers, PER
// lookups per lane per pass (lookups w0 + 64 j + lane of the wave's tile).
template <uint32_t WAVES, uint32_t MODE, bool TIMED, uint32_t PER>
__global__ void __launch_bounds__(64 * WAVES)
    lookup_quad(TableRef T, const uint4 *__restrict__ keys, uint64_t n,
                uint8_t *__restrict__ found, uint64_t *__restrict__ vals) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave0 = ((uint64_t)blockIdx.x * WAVES + (threadIdx.x >> 6)) * 64u * PER;
  const uint64_t stride = (uint64_t)gridDim.x * WAVES * 64u * PER;
  uint4 k[PER];
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    const uint64_t i = wave0 + 64u * j + lane;
    k[j] = i < n ? load_stream(keys + i) : zero4();
  }
  // the wave stays together (the quads exchange registers): the loop runs
  // over the wave's tiles
  for (uint64_t w0 = wave0; w0 < n; w0 += stride) {
    bool ok[PER];
    uint4 kn[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) ok[j] = w0 + 64u * j + lane < n;
    quad_pass<MODE, TIMED, PER>(T, k, ok, found + w0 + lane, vals + w0 + lane, [&] {
#pragma unroll
      for (uint32_t j = 0; j < PER; ++j) {
        const uint64_t i = w0 + stride + 64u * j + lane;
        kn[j] = i < n ? load_stream(keys + i) : zero4();
      }
    });
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) k[j] = kn[j];
  }
}

// One table's batch, one lane per lookup with lines in registers, PER
// lookups per lane per pass (lookups w0 + 64 j + lane of the wave's tile).
template <uint32_t WAVES, uint32_t MODE, bool TIMED, uint32_t PER>
__global__ void __launch_bounds__(64 * WAVES)
    lookup_reg(TableRef T, const uint4 *__restrict__ keys, uint64_t n,
               uint8_t *__restrict__ found, uint64_t *__restrict__ vals) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave0 = ((uint64_t)blockIdx.x * WAVES + (threadIdx.x >> 6)) * 64u * PER;
  const uint64_t stride = (uint64_t)gridDim.x * WAVES * 64u * PER;
  uint4 k[PER];
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    const uint64_t i = wave0 + 64u * j + lane;
    k[j] = i < n ? load_stream(keys + i) : zero4();
  }
  for (uint64_t w0 = wave0; w0 < n; w0 += stride) {
    bool ok[PER];
    uint4 kn[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) ok[j] = w0 + 64u * j + lane < n;
    reg_pass<MODE, TIMED, PER>(T, k, ok, found + w0 + lane, vals + w0 + lane, [&] {
#pragma unroll
      for (uint32_t j = 0; j < PER; ++j) {
        const uint64_t i = w0 + stride + 64u * j + lane;
        kn[j] = i < n ? load_stream(keys + i) : zero4();
      }
    });
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) k[j] = kn[j];
  }
}

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
// LANES = 8: lines land in LDS (the passes of lookup_lds / lookup_dual,
// PER 1 or 2); NB = 2 gives each wave the second line buffer of the
// pessimistic mode, and with NB = 1 the host passes no pessimistic item.
// LANES = 4: lines spread over a quad's registers (the passes of
// lookup_quad, PER 1 or 2, no LDS); NB = 2 compiles in the pessimistic
// mode, whose secondary lines take registers of their own.  LANES = 1: bucket heads in
// registers (the passes of lookup_reg, PER 1, 2 or 4, every mode, no LDS).
template <uint32_t WAVES, uint32_t NB, uint32_t PER, bool DYN, uint32_t LANES>
__global__ void __launch_bounds__(64 * WAVES)
    lookup_plan(const PlanItem *__restrict__ items, uint32_t nitems,
                const uint4 *__restrict__ keys, uint8_t *__restrict__ found,
                uint64_t *__restrict__ vals, uint32_t *__restrict__ ctr) {
  static_assert(LANES == 1 || PER <= 2, "lines in LDS: one or two lookups per lane");
  static_assert(LANES != 4 || PER <= 2, "lines in a quad: one or two lookups per lane");
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
    const TableRef T{I.tab, I.seed, I.log2b};
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
      if constexpr (LANES == 1) {
        if (I.mode == kModeCuckoopp)
          reg_pass<kModeCuckoopp, false, PER>(T, k, ok, found + ia, vals + ia, pre);
        else if (I.mode == kModeOptimistic)
          reg_pass<kModeOptimistic, false, PER>(T, k, ok, found + ia, vals + ia, pre);
        else
          reg_pass<kModeBoth, false, PER>(T, k, ok, found + ia, vals + ia, pre);
      } else if constexpr (LANES == 4) {
        if (I.mode == kModeCuckoopp)
          quad_pass<kModeCuckoopp, false, PER>(T, k, ok, found + ia, vals + ia, pre);
        else if (I.mode == kModeOptimistic)
          quad_pass<kModeOptimistic, false, PER>(T, k, ok, found + ia, vals + ia, pre);
        else if (NB == 2)
          quad_pass<kModeBoth, false, PER>(T, k, ok, found + ia, vals + ia, pre);
      } else if constexpr (PER == 1) {
        if (I.mode == kModeCuckoopp) {
          lds_pass<kModeCuckoopp>(w, T, k[0], ok[0], found + ia, vals + ia, pre);
        } else if (I.mode == kModeOptimistic) {
          lds_pass<kModeOptimistic>(w, T, k[0], ok[0], found + ia, vals + ia, pre);
        } else if (NB == 2) {
          lds_pass<kModeBoth>(w, T, k[0], ok[0], found + ia, vals + ia, pre);
        }
      } else {
        const uint64_t ib = ia + 64u;
        if (I.mode == kModeCuckoopp) {
          dual_pass<kModeCuckoopp>(w, T, k[0], ok[0], k[1], ok[1], found + ia, vals + ia,
                                   found + ib, vals + ib, pre);
        } else if (I.mode == kModeOptimistic) {
          dual_pass<kModeOptimistic>(w, T, k[0], ok[0], k[1], ok[1], found + ia, vals + ia,
                                     found + ib, vals + ib, pre);
        } else if (NB == 2) {
          lds_pass<kModeBoth>(w, T, k[0], ok[0], found + ia, vals + ia, [] {});
          lds_pass<kModeBoth>(w, T, k[1], ok[1], found + ib, vals + ib, pre);
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
    // every ticket this wave will ever take is taken: count the wave out;
    // the last one (which sees every other wave's tickets) rewinds both
    const uint32_t out = __hip_atomic_fetch_add(ctr + 1, 1u, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (out == gridDim.x * WAVES - 1u) {
      __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ctr + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

uint64_t capped_grid(uint64_t n, uint64_t per_block, uint32_t blocks_per_cu, int num_cus) {
  uint64_t grid = (n + per_block - 1) / per_block;
  if (blocks_per_cu) {
    const uint64_t cap = (uint64_t)blocks_per_cu * (uint64_t)num_cus;
    if (grid > cap) grid = cap;
  }
  return grid > 0x7fffffffull ? 0x7fffffffull : grid;
}

template <uint32_t WAVES, uint32_t MODE, bool TIMED, uint32_t PER>
hipError_t launch_reg(const ckpp_table *t, const TableRef &T, const uint4 *keys, uint64_t n,
                      uint8_t *found, uint64_t *vals, hipStream_t s) {
  const uint64_t grid =
      capped_grid(n, 64ull * PER * WAVES, t->lookup_launch.blocks_per_cu, t->num_cus);
  hipLaunchKernelGGL((lookup_reg<WAVES, MODE, TIMED, PER>), dim3((uint32_t)grid),
                     dim3(64 * WAVES), 0, s, T, keys, n, found, vals);
  return hipGetLastError();
}

template <uint32_t WAVES, uint32_t MODE, bool TIMED, uint32_t PER>
hipError_t launch_quad(const ckpp_table *t, const TableRef &T, const uint4 *keys, uint64_t n,
                       uint8_t *found, uint64_t *vals, hipStream_t s) {
  const uint64_t grid =
      capped_grid(n, 64ull * PER * WAVES, t->lookup_launch.blocks_per_cu, t->num_cus);
  hipLaunchKernelGGL((lookup_quad<WAVES, MODE, TIMED, PER>), dim3((uint32_t)grid),
                     dim3(64 * WAVES), 0, s, T, keys, n, found, vals);
  return hipGetLastError();
}

template <uint32_t WAVES, uint32_t MODE, bool TIMED>
hipError_t launch_shape(const ckpp_table *t, const TableRef &T, const uint4 *keys, uint64_t n,
                        uint8_t *found, uint64_t *vals, hipStream_t s) {
  const ckpp_launch_t &L = t->lookup_launch;
  if (L.lanes_per_lookup == 4) {
    if (L.lookups_per_lane == 2)
      return launch_quad<WAVES, MODE, TIMED, 2>(t, T, keys, n, found, vals, s);
    return launch_quad<WAVES, MODE, TIMED, 1>(t, T, keys, n, found, vals, s);
  }
  if (L.lanes_per_lookup == 1) {
    if (L.lookups_per_lane == 4)
      return launch_reg<WAVES, MODE, TIMED, 4>(t, T, keys, n, found, vals, s);
    if (L.lookups_per_lane == 2)
      return launch_reg<WAVES, MODE, TIMED, 2>(t, T, keys, n, found, vals, s);
    return launch_reg<WAVES, MODE, TIMED, 1>(t, T, keys, n, found, vals, s);
  }
  if (MODE != kModeBoth && L.lookups_per_lane == 2) {
    constexpr uint32_t M = MODE == kModeBoth ? kModeCuckoopp : MODE;
    const uint64_t grid = capped_grid(n, 128ull * WAVES, L.blocks_per_cu, t->num_cus);
    hipLaunchKernelGGL((lookup_dual<WAVES, M, TIMED>), dim3((uint32_t)grid), dim3(64 * WAVES), 0,
                       s, T, keys, n, found, vals);
  } else {
    const uint64_t grid = capped_grid(n, 64ull * WAVES, L.blocks_per_cu, t->num_cus);
    hipLaunchKernelGGL((lookup_lds<WAVES, MODE, TIMED>), dim3((uint32_t)grid), dim3(64 * WAVES),
                       0, s, T, keys, n, found, vals);
  }
  return hipGetLastError();
}

template <uint32_t MODE, bool TIMED>
hipError_t launch_mode(const ckpp_table *t, const TableRef &T, const uint4 *keys, uint64_t n,
                       uint8_t *found, uint64_t *vals, hipStream_t s) {
  switch (t->lookup_launch.block) {
    case 64: return launch_shape<1, MODE, TIMED>(t, T, keys, n, found, vals, s);
    case 128: return launch_shape<2, MODE, TIMED>(t, T, keys, n, found, vals, s);
    default: return launch_shape<4, MODE, TIMED>(t, T, keys, n, found, vals, s);
  }
}

template <bool TIMED>
hipError_t launch_timing(const ckpp_table *t, const TableRef &T, const uint4 *keys, uint64_t n,
                         uint32_t mode, uint8_t *found, uint64_t *vals, hipStream_t s) {
  if (mode == kModeBoth) return launch_mode<kModeBoth, TIMED>(t, T, keys, n, found, vals, s);
  if (mode == kModeOptimistic)
    return launch_mode<kModeOptimistic, TIMED>(t, T, keys, n, found, vals, s);
  return launch_mode<kModeCuckoopp, TIMED>(t, T, keys, n, found, vals, s);
}

template <uint32_t WAVES, uint32_t NB, uint32_t PER, uint32_t LANES>
hipError_t launch_plan_shape(const PlanItem *d_items, uint32_t nitems, uint32_t *d_ctr,
                             const ckpp_plan_launch_t &L, int num_cus, const uint4 *keys,
                             uint8_t *found, uint64_t *vals, hipStream_t s) {
  // persistent grid: blocks_per_cu per CU, but no more waves than items
  const uint64_t grid = capped_grid(nitems, WAVES, L.blocks_per_cu, num_cus);
  if (L.schedule == CKPP_PLAN_DYNAMIC)
    hipLaunchKernelGGL((lookup_plan<WAVES, NB, PER, true, LANES>), dim3((uint32_t)grid),
                       dim3(64 * WAVES), 0, s, d_items, nitems, keys, found, vals, d_ctr);
  else
    hipLaunchKernelGGL((lookup_plan<WAVES, NB, PER, false, LANES>), dim3((uint32_t)grid),
                       dim3(64 * WAVES), 0, s, d_items, nitems, keys, found, vals, d_ctr);
  return hipGetLastError();
}

template <uint32_t WAVES>
hipError_t launch_plan_waves(const PlanItem *d_items, uint32_t nitems, uint32_t *d_ctr,
                             bool two_buffers, const ckpp_plan_launch_t &L, int num_cus,
                             const uint4 *keys, uint8_t *found, uint64_t *vals, hipStream_t s) {
  if (L.lanes_per_lookup == 1) {
    if (L.lookups_per_lane == 4)
      return launch_plan_shape<WAVES, 1, 4, 1>(d_items, nitems, d_ctr, L, num_cus, keys, found,
                                               vals, s);
    if (L.lookups_per_lane == 2)
      return launch_plan_shape<WAVES, 1, 2, 1>(d_items, nitems, d_ctr, L, num_cus, keys, found,
                                               vals, s);
    return launch_plan_shape<WAVES, 1, 1, 1>(d_items, nitems, d_ctr, L, num_cus, keys, found,
                                             vals, s);
  }
  if (L.lanes_per_lookup == 4) {
    if (L.lookups_per_lane == 2)
      return two_buffers ? launch_plan_shape<WAVES, 2, 2, 4>(d_items, nitems, d_ctr, L, num_cus,
                                                             keys, found, vals, s)
                         : launch_plan_shape<WAVES, 1, 2, 4>(d_items, nitems, d_ctr, L, num_cus,
                                                             keys, found, vals, s);
    return two_buffers ? launch_plan_shape<WAVES, 2, 1, 4>(d_items, nitems, d_ctr, L, num_cus,
                                                           keys, found, vals, s)
                       : launch_plan_shape<WAVES, 1, 1, 4>(d_items, nitems, d_ctr, L, num_cus,
                                                           keys, found, vals, s);
  }
  if (two_buffers) {
    if (L.lookups_per_lane == 2)
      return launch_plan_shape<WAVES, 2, 2, 8>(d_items, nitems, d_ctr, L, num_cus, keys, found,
                                               vals, s);
    return launch_plan_shape<WAVES, 2, 1, 8>(d_items, nitems, d_ctr, L, num_cus, keys, found,
                                             vals, s);
  }
  if (L.lookups_per_lane == 2)
    return launch_plan_shape<WAVES, 1, 2, 8>(d_items, nitems, d_ctr, L, num_cus, keys, found,
                                             vals, s);
  return launch_plan_shape<WAVES, 1, 1, 8>(d_items, nitems, d_ctr, L, num_cus, keys, found, vals,
                                           s);
}

}  // namespace

hipError_t launch_plan(const PlanItem *d_items, uint32_t nitems, uint32_t *d_ctr, bool two_buffers,
                       const ckpp_plan_launch_t &L, int num_cus, const void *d_keys,
                       uint8_t *d_found, uint64_t *d_values, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  const uint4 *keys = reinterpret_cast<const uint4 *>(d_keys);
  switch (L.block) {
    case 64:
      return launch_plan_waves<1>(d_items, nitems, d_ctr, two_buffers, L, num_cus, keys, d_found,
                                  d_values, s);
    case 128:
      return launch_plan_waves<2>(d_items, nitems, d_ctr, two_buffers, L, num_cus, keys, d_found,
                                  d_values, s);
    default:
      return launch_plan_waves<4>(d_items, nitems, d_ctr, two_buffers, L, num_cus, keys, d_found,
                                  d_values, s);
  }
}

hipError_t launch_lookup(const ckpp_table *t, const void *d_keys, uint64_t n, uint32_t mode,
                         const TimerArgs *timers, uint8_t *d_found, uint64_t *d_values,
                         hipStream_t s) {
  const uint4 *keys = reinterpret_cast<const uint4 *>(d_keys);
  TableRef T{reinterpret_cast<const uint4 *>(t->d_table), t->seed, t->log2_buckets};
  if (!timers) return launch_timing<false>(t, T, keys, n, mode, d_found, d_values, s);
  T.now = timers->now;
  T.refresh = timers->refresh;
  T.expiry = timers->expiry;
  return launch_timing<true>(t, T, keys, n, mode, d_found, d_values, s);
}

}  // namespace ckpp

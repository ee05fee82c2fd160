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
// (lookup_reg).  A plan's persistent kernel over many tables' batches
// (lookup_plan, in ckpp_plan.hip) runs the same passes.  On a table
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

// A batch this small is bound by the latency of one lookup's few
// dependent loads, not by requests: one lane per lookup in 64-thread blocks
// finishes it soonest (measured on MI355X, bursts of 1..2048 lookups on a
// 2^24-bucket table: 21.4 us p50 from submission to completion against
// 25.4 us in the default shape).  Used while no caller set a shape.
constexpr uint64_t kSmallBatch = 4096;

template <uint32_t MODE, bool TIMED>
hipError_t launch_mode(const ckpp_table *t, const TableRef &T, const uint4 *keys, uint64_t n,
                       uint8_t *found, uint64_t *vals, hipStream_t s) {
  if (!t->launch_set && n <= kSmallBatch)
    return launch_reg<1, MODE, TIMED, 1>(t, T, keys, n, found, vals, s);
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

}  // namespace

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

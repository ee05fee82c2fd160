// ckpp_plan.hip -- plans: many tables' lookup batches served by one
// persistent launch.  The kernel (lookup_plan, ckpp_plan_dev.h) runs the
// lookup passes of the one-table kernels over work items; the C ABI below
// cuts the batches into items and launches it.  This unit instantiates the
// kernel without timers, ckpp_plan_timed.hip the one with.

#include <algorithm>
#include <new>
#include <stdint.h>
#include <vector>

#include "ckpp_plan_dev.h"

namespace ckpp {

hipError_t launch_plan(const PlanItem *d_items, uint32_t nitems, uint32_t *d_ctr, bool two_buffers,
                       const TimerArgs *timers, const ckpp_plan_launch_t &L, int num_cus,
                       const void *d_keys, uint8_t *d_found, uint64_t *d_values, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  PlanArgs A{d_items, nitems, reinterpret_cast<const uint4 *>(d_keys), d_found, d_values, d_ctr,
             TimerArgs{0u, 0u, 0u}};
  if (!timers) return launch_plan_block<false>(A, two_buffers, L, num_cus, s);
  A.tm = *timers;
  return launch_plan_timed(A, two_buffers, L, num_cus, s);
}

}  // namespace ckpp

using ckpp::DeviceGuard;
using ckpp::dev_status;
using ckpp::PlanItem;

struct ckpp_plan {
  int device;
  int num_cus;
  uint32_t ntables;
  bool two_buffers;  // some table uses the pessimistic mode
  bool timed;        // some table has timers
  uint64_t lookups;
  uint64_t key_span;
  std::vector<uint64_t> offsets, counts;
  std::vector<PlanItem> tables;  // per table: its parameters (start, count unused)
  PlanItem *d_items;
  uint32_t nitems;
  uint32_t *d_ctr;  // next item, finished waves
  ckpp_plan_launch_t launch;
};

namespace {

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool valid_launch(const ckpp_plan_launch_t &L) {
  const bool lanes_ok =
      L.lanes_per_lookup == 1 || L.lanes_per_lookup == 4 || L.lanes_per_lookup == 8;
  const bool per_ok = L.lookups_per_lane == 1 || L.lookups_per_lane == 2 ||
                      (L.lookups_per_lane == 4 && L.lanes_per_lookup == 1);
  return lanes_ok && per_ok &&
         (L.block == 64 || L.block == 128 || L.block == 256) && L.blocks_per_cu >= 1 &&
         L.blocks_per_cu <= 64 && L.passes_per_item >= 1 && L.passes_per_item <= 64 &&
         (L.schedule == CKPP_PLAN_STATIC || L.schedule == CKPP_PLAN_DYNAMIC);
}

// Cuts every batch into items of at most `tile` lookups, table by table.
int build_items(ckpp_plan *p, const ckpp_plan_launch_t &L) {
  const uint64_t tile = (uint64_t)L.passes_per_item * 64u * L.lookups_per_lane;
  std::vector<PlanItem> items;
  for (uint32_t i = 0; i < p->ntables; ++i) {
    for (uint64_t o = 0; o < p->counts[i]; o += tile) {
      const uint64_t c = std::min(tile, p->counts[i] - o);
      PlanItem it = p->tables[i];
      it.start = p->offsets[i] + o;
      it.count = (uint32_t)c;
      items.push_back(it);
      if (items.size() > 0x7fffffffull) return CKPP_EINVAL;
    }
  }
  PlanItem *d = nullptr;
  if (!items.empty()) {
    hipError_t e = hipMalloc(&d, items.size() * sizeof(PlanItem));
    if (e != hipSuccess) return dev_status(e);
    e = hipMemcpy(d, items.data(), items.size() * sizeof(PlanItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return dev_status(e);
    }
  }
  if (p->d_items) {
    (void)hipDeviceSynchronize();
    (void)hipFree(p->d_items);
  }
  p->d_items = d;
  p->nitems = (uint32_t)items.size();
  p->launch = L;
  return CKPP_OK;
}

void free_plan(ckpp_plan *p) {
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_ctr) (void)hipFree(p->d_ctr);
  delete p;
}

int plan_lookup(ckpp_plan *p, const void *d_keys, uint8_t *d_found, uint64_t *d_values,
                const ckpp::TimerArgs *tm, void *stream) {
  if (p->nitems == 0) return CKPP_OK;
  if (!d_keys || !d_found || !d_values) return CKPP_EINVAL;
  if (!aligned(d_keys, 16) || !aligned(d_values, 8)) return CKPP_EINVAL;
  DeviceGuard g(p->device);
  if (!g.ok()) return CKPP_EDEVICE;
  return dev_status(ckpp::launch_plan(p->d_items, p->nitems, p->d_ctr, p->two_buffers, tm,
                                      p->launch, p->num_cus, d_keys, d_found, d_values,
                                      reinterpret_cast<hipStream_t>(stream)));
}


}  // namespace

extern "C" {

int ckpp_plan_create(ckpp_plan **out, ckpp_table *const *tables, uint32_t ntables,
                     const uint64_t *h_offsets, const uint64_t *h_counts,
                     const uint32_t *h_modes) {
  if (!out) return CKPP_EINVAL;
  *out = nullptr;
  if (!tables || ntables == 0 || !h_offsets || !h_counts) return CKPP_EINVAL;
  std::vector<PlanItem> desc(ntables);
  std::vector<uint32_t> order(ntables);
  bool two = false, any_timed = false;
  uint64_t lookups = 0, span = 0;
  for (uint32_t i = 0; i < ntables; ++i) {
    const ckpp_table *t = tables[i];
    if (!t || t->device != tables[0]->device) return CKPP_EINVAL;
    uint32_t mode = h_modes ? h_modes[i] : (uint32_t)CKPP_LOOKUP_DEFAULT;
    if (mode > CKPP_LOOKUP_OPTIMISTIC) return CKPP_EINVAL;
    // a plain table keeps no filter: its default lookup reads both buckets
    if (mode == CKPP_LOOKUP_DEFAULT && (t->flags & CKPP_PLAIN)) mode = CKPP_LOOKUP_BOTH;
    two = two || mode == CKPP_LOOKUP_BOTH;
    if (h_counts[i] > (1ull << 40) || h_offsets[i] > (1ull << 40)) return CKPP_EINVAL;
    const bool tm = (t->flags & CKPP_TIMERS) != 0u;
    any_timed = any_timed || tm;
    desc[i] = PlanItem{reinterpret_cast<const uint4 *>(t->d_table), t->seed, 0ull, 0u,
                       t->log2_buckets, mode | (tm ? ckpp::kPlanItemTimed : 0u), i};
    lookups += h_counts[i];
    span = std::max(span, h_offsets[i] + h_counts[i]);
    order[i] = i;
  }
  // the ranges must be disjoint
  std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    return h_offsets[a] < h_offsets[b];
  });
  uint64_t end = 0;
  for (uint32_t i : order) {
    if (h_counts[i] == 0) continue;
    if (h_offsets[i] < end) return CKPP_EINVAL;
    end = h_offsets[i] + h_counts[i];
  }
  DeviceGuard g(tables[0]->device);
  if (!g.ok()) return CKPP_EDEVICE;
  ckpp_plan *p = new (std::nothrow) ckpp_plan();
  if (!p) return CKPP_ENOMEM;
  p->device = tables[0]->device;
  p->num_cus = tables[0]->num_cus;
  p->ntables = ntables;
  p->two_buffers = two;
  p->timed = any_timed;
  p->lookups = lookups;
  p->key_span = span;
  p->offsets.assign(h_offsets, h_offsets + ntables);
  p->counts.assign(h_counts, h_counts + ntables);
  p->tables = desc;
  p->d_items = nullptr;
  p->d_ctr = nullptr;
  p->nitems = 0;
  hipError_t e = hipMalloc(&p->d_ctr, 256);
  if (e == hipSuccess) e = hipMemset(p->d_ctr, 0, 256);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_plan(p);
    return dev_status(e);
  }
  const ckpp_plan_launch_t L{1u, 128u, 8u, 1u, CKPP_PLAN_STATIC, 8u};
  const int rc = build_items(p, L);
  if (rc != CKPP_OK) {
    free_plan(p);
    return rc;
  }
  *out = p;
  return CKPP_OK;
}

int ckpp_plan_destroy(ckpp_plan *p) {
  if (!p) return CKPP_OK;
  DeviceGuard g(p->device);
  (void)hipDeviceSynchronize();
  free_plan(p);
  return CKPP_OK;
}


int ckpp_plan_lookup(ckpp_plan *p, const void *d_keys, uint8_t *d_found, uint64_t *d_values,
                     void *stream) {
  if (!p || p->timed) return CKPP_EINVAL;
  return plan_lookup(p, d_keys, d_found, d_values, nullptr, stream);
}

int ckpp_plan_lookup_at(ckpp_plan *p, const void *d_keys, uint8_t *d_found, uint64_t *d_values,
                        uint16_t now, uint32_t refresh, uint16_t expiry, void *stream) {
  if (!p || !p->timed || refresh > 1u) return CKPP_EINVAL;
  if (refresh && !ckpp::in_window(expiry, now)) return CKPP_EINVAL;
  const ckpp::TimerArgs tm{now, refresh, expiry};
  return plan_lookup(p, d_keys, d_found, d_values, &tm, stream);
}

int ckpp_plan_set_launch(ckpp_plan *p, const ckpp_plan_launch_t *cfg) {
  if (!p || !cfg || !valid_launch(*cfg)) return CKPP_EINVAL;
  DeviceGuard g(p->device);
  if (!g.ok()) return CKPP_EDEVICE;
  return build_items(p, *cfg);
}

int ckpp_plan_get_launch(const ckpp_plan *p, ckpp_plan_launch_t *cfg) {
  if (!p || !cfg) return CKPP_EINVAL;
  *cfg = p->launch;
  return CKPP_OK;
}

int ckpp_plan_info(const ckpp_plan *p, ckpp_plan_info_t *out) {
  if (!p || !out) return CKPP_EINVAL;
  out->ntables = p->ntables;
  out->nitems = p->nitems;
  out->lookups = p->lookups;
  out->key_span = p->key_span;
  return CKPP_OK;
}

}  // extern "C"

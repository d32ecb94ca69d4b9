// Batched form of the filter: the launch schedule of many jobs.
//
// Every pass of the per-job sequence (down(0) .. down(L-2), then up(L-2) ..
// up(0)) is run for all jobs that have it as one launch per kernel class; the
// classes are the K loop (exact 4, 8, 16 or guarded 8, 16, 32), the boost map,
// whether the job's level l takes the fused form, and for the product-sum up(l)
// whether level l + 1 is the job's top; the one-plane collapses of the fused
// levels depend on neither K nor the map and share one launch.  Passes are
// aligned on the level index l, so a job with fewer levels simply sits out the
// coarse passes: each job still sees its own passes in its own order, and the
// kernels are the per-job wave bodies, so a job's result does not depend on the
// batch.
//
// The launches find their jobs in a table at the start of the workspace: per
// launch, the argument records of its jobs and the prefix sums of their wave
// counts (a wave finds its job by binary search).
//
// A serving step uses the same launches for independent passes of different
// jobs: passes of one kernel class share a launch whatever their level.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include "fllf_kernels.h"

namespace fllf {

const char *const kBatchDownNames[kMaxLevels] = {
    "bdown_l0", "bdown_l1", "bdown_l2",  "bdown_l3",  "bdown_l4",  "bdown_l5",  "bdown_l6",  "bdown_l7",
    "bdown_l8", "bdown_l9", "bdown_l10", "bdown_l11", "bdown_l12", "bdown_l13", "bdown_l14", "bdown_l15"};
const char *const kBatchUpNames[kMaxLevels] = {
    "bup_l0", "bup_l1", "bup_l2",  "bup_l3",  "bup_l4",  "bup_l5",  "bup_l6",  "bup_l7",
    "bup_l8", "bup_l9", "bup_l10", "bup_l11", "bup_l12", "bup_l13", "bup_l14", "bup_l15"};

Tuning default_tuning(fllf_storage storage) {
  // Autotuned on the 3840x2160 RGB K = 8 workload.  The level-0 passes want
  // many short segments; the float32 down passes that read a level of records
  // (one wave per SIMD) want long ones.
  Tuning t;
  t.p[kTuneDown0] = 12288;
  t.p[kTuneDown] = storage == FLLF_STORE_F32 ? 512 : 1536;
  t.p[kTuneUp0] = 12288;  // up(0) with the level-1 collapse folded in wants short segments
  // up(l >= 1) is the one-plane collapse on the large levels: little work per
  // row, so short segments (many waves) hide the row latency
  t.p[kTuneUp] = 12288;
  t.p[kTuneGridCap] = 0;
  // non-temporal stores in down(0) and up(0): the level-1 records down(0)
  // writes (the largest plane) then go to HBM without passing through the MALL,
  // and down(1) reads them back faster (4K RGB K = 8 float32: down_l1 145 ->
  // 119 us, down_l0 102 -> 104 us, the step 470 -> 440 us; float16 332 -> 327 us)
  t.p[kTuneNtStores] = (1 << kNtDown0) | (1 << kNtUp0);
  return t;
}

namespace {

int pair_dwords(fllf_storage s) { return s == FLLF_STORE_F32 ? 2 : 1; }

// Waves of pass down(l) / up(l) of one job (the same geometry the launch uses).
uint32_t pass_waves(const JobPlan &P, int l, bool down, const Tuning &tu) {
  return (uint32_t)geom_waves(pass_geom(P, l, down, tu));
}

// Appends to the table `out->blob` (growing it) one launch per kernel class of
// the given (job, pass) items.  Items of one class may be at different levels:
// down(l >= 1) passes of any level share a kernel, as do up(l >= 1) passes, and
// the collapses of all fused levels share one launch.
void add_launches(const PassItem *items, int n, int dwp, char *ws, const Tuning &tu0, BatchSchedule *out) {
  // n jobs share each launch of the pass, so every job aims at fewer waves
  // (longer segments, less halo): every segment target scales with 1/sqrt(n),
  // down to 256 waves a job.  Without it a small job's down(l >= 1) would run
  // one- to four-row segments that read its records 1.75 to 4 times (64-image
  // batch with the level >= 1 down target scaled too: float32 6.37 -> 6.26 ms,
  // float16 4.36 -> 4.07 ms).  Results do not depend on the launch shape.
  Tuning tu = tu0;
  if (n > 1) {
    const double f = 1.0 / std::sqrt((double)n);
    for (int k : {kTuneDown0, kTuneDown, kTuneUp0, kTuneUp}) tu.p[k] = std::max(256, (int)(tu0.p[k] * f));
  }
  size_t off = out->blob.size();
  auto reserve = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    out->blob.resize(off, 0);
    return at;
  };
  // (kind, level-0 pass, K loop, exact, map, has O_{l+1}, fused level)
  typedef std::tuple<int, bool, int, bool, bool, bool, bool> Key;
  std::map<Key, std::vector<int>> groups;
  for (int i = 0; i < n; ++i) {
    const PassItem &it = items[i];
    if (it.P->levels == 1) {
      BatchLaunch b{};
      b.kind = 2;
      b.copy = it.P->copy;
      b.bytes = 2.0 * (double)(it.P->lv[0].n * it.P->C * sizeof(float));
      out->launches.push_back(b);
      continue;
    }
    int km;
    bool ex;
    k_class(it.P->K, &km, &ex);
    const bool hasd = !it.down && it.l + 1 < it.P->levels - 1;
    if (!it.down && it.l == 1 && fold_level1(*it.P)) continue;  // done inside up(0)
    // fused level l; for up(0), whether the level-1 collapse is folded in
    const bool fuse = !it.down && it.l == 0 ? fold_level1(*it.P) : fused_level(*it.P, it.l);
    if (!it.down && it.l >= 1 && fuse)  // the collapse: one kernel for every job
      groups[Key(1, false, 0, false, false, false, true)].push_back(i);
    else
      groups[Key(it.down ? 0 : 1, it.l == 0, km, ex, it.P->m_map != nullptr || it.P->s_map != nullptr, hasd, fuse)]
          .push_back(i);
  }
  for (auto &kv : groups) {
    const std::vector<int> &is = kv.second;
    BatchLaunch b{};
    b.kind = std::get<0>(kv.first);
    const bool down = b.kind == 0;
    b.l0 = std::get<1>(kv.first);
    b.km = std::get<2>(kv.first);
    b.ex = std::get<3>(kv.first);
    b.map = std::get<4>(kv.first);
    b.hasd = std::get<5>(kv.first);
    b.fuse = std::get<6>(kv.first);
    b.level = items[is[0]].l;  // the finest level of the group names the launch
    for (int i : is) b.level = std::min(b.level, items[i].l);
    b.njobs = (int)is.size();
    const size_t rec = down ? sizeof(DownArgs) : sizeof(UpArgs);
    b.args_off = reserve(rec * is.size());
    b.start_off = reserve(sizeof(uint32_t) * (is.size() + 1));
    uint32_t total = 0;
    for (size_t q = 0; q < is.size(); ++q) {
      const PassItem &it = items[is[q]];
      std::memcpy(out->blob.data() + b.start_off + 4 * q, &total, 4);
      total += pass_waves(*it.P, it.l, down, tu);
      b.bytes += down ? down_bytes(*it.P, it.l, dwp) : up_bytes(*it.P, it.l, dwp);
      if (ws) {
        if (down) {
          const DownArgs a = make_down_args(*it.P, it.l, ws, dwp, tu);
          std::memcpy(out->blob.data() + b.args_off + rec * q, &a, rec);
        } else {
          UpArgs a = make_up_args(*it.P, it.l, ws, dwp, tu);
          if (b.fuse && !b.l0 && !a.oc) a.oc = a.gc;  // the collapse expands G_{l+1} at the top
          std::memcpy(out->blob.data() + b.args_off + rec * q, &a, rec);
        }
      }
    }
    std::memcpy(out->blob.data() + b.start_off + 4 * is.size(), &total, 4);
    b.waves = total;
    out->launches.push_back(b);
  }
  out->table_bytes = off;
}

}  // namespace

void build_step(const PassItem *items, int n, fllf_storage storage, char *ws, const Tuning &tu,
                BatchSchedule *out) {
  out->launches.clear();
  out->blob.clear();
  add_launches(items, n, pair_dwords(storage), ws, tu, out);
}

void build_batch(const JobPlan *P, int n, fllf_storage storage, char *ws, const Tuning &tu, BatchSchedule *out) {
  out->launches.clear();
  out->blob.clear();
  out->table_bytes = 0;
  const int dwp = pair_dwords(storage);
  int maxL = 1;
  std::vector<PassItem> items;
  for (int j = 0; j < n; ++j) {
    maxL = std::max(maxL, P[j].levels);
    if (P[j].levels == 1) items.push_back(PassItem{&P[j], 0, true});
  }
  add_launches(items.data(), (int)items.size(), dwp, ws, tu, out);
  // passes aligned on the level index: every job's down passes before its up passes
  for (int pass = 0; pass < 2 * (maxL - 1); ++pass) {
    const bool down = pass < maxL - 1;
    const int l = down ? pass : 2 * (maxL - 1) - 1 - pass;
    items.clear();
    for (int j = 0; j < n; ++j)
      if (l + 1 < P[j].levels) items.push_back(PassItem{&P[j], l, down});
    add_launches(items.data(), (int)items.size(), dwp, ws, tu, out);
  }
}

size_t step_table_bound(int n) {
  // per launch group: the records and n_g + 1 offsets, each padded to kAlign;
  // groups: down 6 K loops x 2 maps x (level 0, separate, fused) = 36, up
  // 6 x 2 x 2 top flags x (level 0, separate) = 48, up(0) with the level-1
  // collapse folded in 6 x 2 = 12, and the collapse
  const size_t groups = 97;
  const size_t rec = std::max(sizeof(DownArgs), sizeof(UpArgs));
  return align_up(rec * (size_t)n + 4 * (size_t)n + groups * (4 + 2 * (kAlign - 1)));
}

size_t batch_table_bytes(const JobPlan *plans, int n, fllf_storage storage) {
  if (n <= 1) return 0;
  BatchSchedule s;
  build_batch(plans, n, storage, nullptr, default_tuning(storage), &s);
  return s.table_bytes;
}

hipError_t launch_batch(const BatchSchedule &s, fllf_storage storage, char *ws, hipStream_t st, LaunchHook *h,
                        const Tuning &tu) {
  switch (storage) {
    case FLLF_STORE_F16: return launch_batch_f16(s, ws, st, h, tu);
    case FLLF_STORE_BF16: return launch_batch_bf16(s, ws, st, h, tu);
    default: return launch_batch_f32(s, ws, st, h, tu);
  }
}

}  // namespace fllf

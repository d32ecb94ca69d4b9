// Batched form of the filter: the launch schedule of many jobs.
//
// Every pass of the per-job sequence (down(0) .. down(L-2), then up(L-2) ..
// up(0)) is run for all jobs that have it as one launch per kernel class; the
// classes are the K loop (exact 4, 8, 16 or guarded 8, 16, 32), the boost map,
// and for up(l) whether level l + 1 is the job's top.  Passes are aligned on
// the level index l, so a job with fewer levels simply sits out the coarse
// passes: each job still sees its own passes in its own order, and the kernels
// are the per-job wave bodies, so a job's result does not depend on the batch.
//
// The launches find their jobs in a table at the start of the workspace: per
// launch, the argument records of its jobs and the prefix sums of their wave
// counts (a wave finds its job by binary search).
#include <algorithm>
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

Tuning default_tuning() {
  // Measured on the 3840x2160 RGB K = 8 workload: the level-0 passes read
  // little per fine row and want many short segments, the passes that read a
  // level of (C, S) records want long ones.
  Tuning t;
  t.p[kTuneDown0] = 12288;
  t.p[kTuneDown] = 1536;
  t.p[kTuneUp0] = 12288;
  t.p[kTuneUp] = 1536;
  t.p[kTuneGridCap] = 0;
  return t;
}

namespace {

int pair_dwords(fllf_storage s) { return s == FLLF_STORE_F32 ? 2 : 1; }

// Waves of pass down(l) / up(l) of one job (the same geometry the launch uses).
uint32_t pass_waves(const JobPlan &P, int l, bool down, const Tuning &tu) {
  const int kind = down ? (l == 0 ? kTuneDown0 : kTuneDown) : (l == 0 ? kTuneUp0 : kTuneUp);
  const Geom g = make_geom(P.lv[l], P.lv[l + 1], P.C, pick_segment(P.lv[l + 1], P.C, tu.p[kind]));
  return (uint32_t)geom_waves(g);
}

// Class of a job's launch: (K loop, exact, map, has O_{l+1}).
typedef std::tuple<int, bool, bool, bool> ClassKey;

}  // namespace

void build_batch(const JobPlan *P, int n, fllf_storage storage, char *ws, const Tuning &tu, BatchSchedule *out) {
  out->launches.clear();
  out->blob.clear();
  const int dwp = pair_dwords(storage);
  int maxL = 1;
  for (int j = 0; j < n; ++j) maxL = std::max(maxL, P[j].levels);
  size_t off = 0;
  auto reserve = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    out->blob.resize(off, 0);
    return at;
  };
  for (int j = 0; j < n; ++j) {
    if (P[j].levels != 1) continue;
    BatchLaunch b{};
    b.kind = 2;
    b.copy_src = P[j].in;
    b.copy_dst = P[j].out;
    b.copy_bytes = P[j].lv[0].n * P[j].C * sizeof(float);
    b.bytes = 2.0 * b.copy_bytes;
    out->launches.push_back(b);
  }
  for (int pass = 0; pass < 2 * (maxL - 1); ++pass) {
    const bool down = pass < maxL - 1;
    const int l = down ? pass : 2 * (maxL - 1) - 1 - pass;
    std::map<ClassKey, std::vector<int>> groups;
    for (int j = 0; j < n; ++j) {
      if (l + 1 >= P[j].levels) continue;
      int km;
      bool ex;
      k_class(P[j].K, &km, &ex);
      const bool hasd = !down && l + 1 < P[j].levels - 1;
      groups[ClassKey(km, ex, P[j].m_map != nullptr, hasd)].push_back(j);
    }
    for (auto &kv : groups) {
      const std::vector<int> &js = kv.second;
      BatchLaunch b{};
      b.kind = down ? 0 : 1;
      b.level = l;
      b.l0 = l == 0;
      b.km = std::get<0>(kv.first);
      b.ex = std::get<1>(kv.first);
      b.map = std::get<2>(kv.first);
      b.hasd = std::get<3>(kv.first);
      b.njobs = (int)js.size();
      const size_t rec = down ? sizeof(DownArgs) : sizeof(UpArgs);
      b.args_off = reserve(rec * js.size());
      b.start_off = reserve(sizeof(uint32_t) * (js.size() + 1));
      uint32_t total = 0;
      for (size_t i = 0; i < js.size(); ++i) {
        const JobPlan &J = P[js[i]];
        std::memcpy(out->blob.data() + b.start_off + 4 * i, &total, 4);
        total += pass_waves(J, l, down, tu);
        b.bytes += down ? down_bytes(J, l, dwp) : up_bytes(J, l, dwp);
        if (ws) {
          if (down) {
            const DownArgs a = make_down_args(J, l, ws, dwp, tu);
            std::memcpy(out->blob.data() + b.args_off + rec * i, &a, rec);
          } else {
            const UpArgs a = make_up_args(J, l, ws, dwp, tu);
            std::memcpy(out->blob.data() + b.args_off + rec * i, &a, rec);
          }
        }
      }
      std::memcpy(out->blob.data() + b.start_off + 4 * js.size(), &total, 4);
      b.waves = total;
      out->launches.push_back(b);
    }
  }
  out->table_bytes = off;
}

size_t batch_table_bytes(const JobPlan *plans, int n, fllf_storage storage) {
  if (n <= 1) return 0;
  BatchSchedule s;
  build_batch(plans, n, storage, nullptr, default_tuning(), &s);
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

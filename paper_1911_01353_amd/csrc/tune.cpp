// Autotuner: picks, per width group, the correlation kernel configuration
// (FFT segment length and templates per workgroup, or the split-BF16 MFMA
// path) that is fastest per output point on this device. Each candidate runs
// on probe templates of the group (their bank built in caller scratch) over
// the first bins of the caller's spectrum and is timed with HIP events. The
// probe is large enough to rank candidates as a full search does: up to 256
// templates over up to 2^20 bins give every candidate thousands of workgroups
// (the long segments and the large blocks included) and write a 2 GiB plane, far
// more than the device's last-level cache holds, so stores cost what they cost
// in a real search; each candidate is timed over rounds of back-to-back launches,
// since single probe launches vary by more than the candidates differ. (A
// 32-template probe over 2^20 bins wrote 256 MiB and favoured 512-point segments
// for groups where 2048-point segments are faster at full size; a 64-template
// one could not rank block sizes.)
// Results are cached per process, keyed by everything that determines them,
// so a plan with the same group widths tunes once and a cached choice never
// changes within the process.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "jerk_internal.h"

namespace jerk {
namespace {

constexpr int32_t kProbeMembers = 256;
constexpr int64_t kProbeBins = 1 << 20;
constexpr int kRounds = 3;
constexpr int kLaunchesPerRound = 4;
constexpr int32_t kSegs[4] = {512, 1024, 2048, 4096};
constexpr int32_t kTpbs[5] = {4, 8, 16, 32, 64};
// Fewer than 8 templates per block pays only where a group's launch is too small to fill the
// device (small searches: more, smaller workgroups); on full-size groups it only adds forward
// transforms and spectrum reads, which the probe does not show. So 4 is tried only
// when the whole group at 8 templates per block gives fewer than 4 waves per SIMD (4 SIMDs per
// compute unit).
constexpr int64_t kFillWavesPerCu = 4 * 4;

struct Cand {
  int32_t path, seg, tpb, ept;
};
// (device ordinal, taps, probe members, probe bins, allow MFMA, group members, bins)
//   -> seconds per output point per candidate
using Key = std::tuple<int, int32_t, int32_t, int64_t, bool, int32_t, int64_t>;
std::mutex g_mu;
std::map<Key, std::vector<std::pair<Cand, double>>> g_cache;

struct Scratch {
  int32_t* members_t;   // probe template indices (for tap generation)
  int32_t* members_out; // 0..m-1 (output rows)
  double2* taps;
  float2* spec_fft;     // [m][2][4096]
  void* frags;
  float2* tw[4];
  float* plane;
  size_t bytes;
};

size_t frag_bytes_max(int32_t max_taps) { return gemm_bank_bytes(kProbeMembers, std::min(512, max_taps), JERK_PATH_GEMM_SPLIT_BF16); }

Scratch layout(const Plan& p, int64_t probe_bins, char* base) {
  Scratch s{};
  size_t off = 0;
  auto take = [&](size_t n) {
    const size_t o = off;
    off = align_up(off + n);
    return base ? base + o : nullptr;
  };
  const int32_t kmax = std::max(16, (p.max_taps + 15) / 16 * 16);
  s.members_t = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * kProbeMembers));
  s.members_out = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * kProbeMembers));
  s.taps = reinterpret_cast<double2*>(take((size_t)kProbeMembers * 2 * kmax * 16));
  s.spec_fft = reinterpret_cast<float2*>(take((size_t)kProbeMembers * 2 * 4096 * 8));
  s.frags = take(frag_bytes_max(kmax));
  for (int i = 0; i < 4; ++i) s.tw[i] = reinterpret_cast<float2*>(take((size_t)kSegs[i] * 8));
  s.plane = reinterpret_cast<float*>(take((size_t)kProbeMembers * 2 * probe_bins * 4));
  s.bytes = off;
  return s;
}

int64_t probe_bins_of(int64_t nbins) { return std::min<int64_t>(nbins, kProbeBins); }

}  // namespace

size_t autotune_scratch_bytes(const Plan& p, int64_t nbins) {
  return layout(p, probe_bins_of(nbins), nullptr).bytes;
}

void autotune(Plan& p, const void* d_spec, int64_t nbins, void* d_scratch, size_t scratch_bytes, uint32_t flags,
              hipStream_t stream) {
  require(d_spec != nullptr && nbins >= 1, JERK_EINVAL, "probe spectrum must be set and nbins >= 1");
  require((flags & ~JERK_TUNE_UNIFORM) == 0, JERK_EINVAL, "unknown flags");
  const int64_t pb = probe_bins_of(nbins);
  require(d_scratch != nullptr && scratch_bytes >= autotune_scratch_bytes(p, nbins), JERK_ENOMEM,
          "scratch smaller than jerk_autotune_scratch_bytes");
  require(reinterpret_cast<uintptr_t>(d_scratch) % 256 == 0, JERK_EINVAL, "scratch must be 256-byte aligned");
  const bool uniform = (flags & JERK_TUNE_UNIFORM) != 0;
  const bool allow_gemm = p.desc.path == JERK_PATH_AUTO && !uniform;
  if (p.desc.path == JERK_PATH_GEMM_SPLIT_BF16 || p.desc.path == JERK_PATH_GEMM_FP16) return;  // nothing to choose
  int dev = 0, n_cu = 0;
  JERK_HIP_CHECK(hipGetDevice(&dev));
  JERK_HIP_CHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t fill_waves = kFillWavesPerCu * std::max(1, n_cu);
  Scratch s = layout(p, pb, static_cast<char*>(d_scratch));
  for (int i = 0; i < 4; ++i) gen_twiddles(s.tw[i], kSegs[i], stream);
  std::vector<int32_t> out_idx(kProbeMembers);
  for (int32_t i = 0; i < kProbeMembers; ++i) out_idx[i] = i;
  JERK_HIP_CHECK(hipMemcpyAsync(s.members_out, out_idx.data(), sizeof(int32_t) * kProbeMembers,
                                hipMemcpyHostToDevice, stream));
  hipEvent_t e0, e1;
  JERK_HIP_CHECK(hipEventCreate(&e0));
  JERK_HIP_CHECK(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};

  std::vector<std::vector<std::pair<Cand, double>>> per_group(p.groups.size());
  for (size_t gi = 0; gi < p.groups.size(); ++gi) {
    const Group& g = p.groups[gi];
    const int32_t m = std::min<int32_t>((int32_t)g.members.size(), kProbeMembers);
    const Key key{dev, g.taps, m, pb, allow_gemm, (int32_t)g.members.size(), nbins};
    {
      std::lock_guard<std::mutex> lock(g_mu);
      auto it = g_cache.find(key);
      if (it != g_cache.end()) {
        per_group[gi] = it->second;
        continue;
      }
    }
    // probe templates: spread over the group (widest and narrowest members included)
    std::vector<int32_t> probe(m);
    for (int32_t i = 0; i < m; ++i)
      probe[i] = g.members[m > 1 ? (size_t)i * (g.members.size() - 1) / (m - 1) : 0];
    JERK_HIP_CHECK(hipMemcpyAsync(s.members_t, probe.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, stream));
    JERK_HIP_CHECK(hipStreamSynchronize(stream));  // `probe` is host stack memory
    taps_launch(p, g.taps, s.members_t, m, s.taps, stream);

    std::vector<Cand> cands;
    for (int32_t seg : kSegs)
      if (seg >= 2 * g.taps)
        for (int32_t ept : {8, 16})
          if (fft_variant_supported(seg, ept))
            for (int32_t tpb : kTpbs) {
              const int64_t n_seg = (nbins + (seg - g.taps + 1) - 1) / (seg - g.taps + 1);
              const int64_t waves8 = n_seg * (((int64_t)g.members.size() + 7) / 8) * (seg / ept / 64);
              if (tpb < 8 && waves8 >= fill_waves) continue;
              cands.push_back({JERK_PATH_FFT_FP32, seg, tpb, ept});
            }
    if (allow_gemm && g.taps <= 512) cands.push_back({JERK_PATH_GEMM_SPLIT_BF16, 0, 0, 0});
    std::vector<std::pair<Cand, double>> res;
    for (const Cand& c : cands) {
      auto run = [&]() {
        if (c.path == JERK_PATH_FFT_FP32) {
          FftJob j{};
          j.spec = static_cast<const float2*>(d_spec);
          j.nbins = pb;
          j.bank_fft = s.spec_fft;
          j.members = s.members_out;
          j.m_begin = 0;
          j.m_end = m;
          j.t_begin = 0;
          j.taps = g.taps;
          j.tpb = c.tpb;
          j.plane = s.plane;
          j.ld = 2 * pb;
          fft_correlate_launch(j, c.seg, c.ept, s.tw[tw_slot(c.seg)], stream);
        } else {
          GemmArgs a{};
          a.spec = static_cast<const float2*>(d_spec);
          a.nbins = pb;
          a.bank_gemm = s.frags;
          a.members = s.members_out;
          a.m_begin = 0;
          a.m_end = m;
          a.t_begin = 0;
          a.t_end = m;
          a.plane = s.plane;
          a.ld = 2 * pb;
          a.taps = g.taps;
          a.path = c.path;
          gemm_correlate_launch(a, stream);
        }
      };
      if (c.path == JERK_PATH_FFT_FP32) {
        fft_spectra_launch(s.taps, m, g.taps, c.seg, s.spec_fft, stream);
      } else {
        Group tmp;
        tmp.taps = g.taps;
        tmp.path = c.path;
        tmp.members.resize(m);
        tmp.gemm_bytes = gemm_bank_bytes(m, g.taps, c.path);
        gemm_bank_build(p, tmp, s.taps, s.frags, stream);
      }
      run();  // warm-up
      // the fastest of a few timed rounds of back-to-back launches: a single probe launch lasts
      // well under a millisecond and varies by tens of percent, more than the candidates differ;
      // a round keeps the device busy, and a round slowed by anything else does not decide
      float best_ms = 0.f;
      for (int r = 0; r < kRounds; ++r) {
        JERK_HIP_CHECK(hipEventRecord(e0, stream));
        for (int l = 0; l < kLaunchesPerRound; ++l) run();
        JERK_HIP_CHECK(hipEventRecord(e1, stream));
        JERK_HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        JERK_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (r == 0 || ms < best_ms) best_ms = ms;
      }
      res.push_back({c, (double)best_ms * 1e-3 / kLaunchesPerRound / ((double)m * 2.0 * (double)pb)});
    }
    {
      std::lock_guard<std::mutex> lock(g_mu);
      g_cache.emplace(key, res);
    }
    per_group[gi] = std::move(res);
  }

  JERK_HIP_CHECK(hipStreamSynchronize(stream));
  if (uniform) {
    // one segment length for all groups: least total estimated time
    int32_t best_seg = 0, best_ept = 0;
    double best_total = 0.0;
    for (int32_t seg : kSegs)
      for (int32_t ept : {8, 16}) {
        if (!fft_variant_supported(seg, ept)) continue;
        double total = 0.0;
        bool ok = true;
        for (size_t gi = 0; gi < p.groups.size() && ok; ++gi) {
          double bt = -1.0;
          for (auto& r : per_group[gi])
            if (r.first.path == JERK_PATH_FFT_FP32 && r.first.seg == seg && r.first.ept == ept &&
                (bt < 0 || r.second < bt))
              bt = r.second;
          if (bt < 0) ok = false;
          else total += bt * (double)p.groups[gi].members.size();
        }
        if (ok && (best_seg == 0 || total < best_total)) {
          best_seg = seg;
          best_ept = ept;
          best_total = total;
        }
      }
    require(best_seg != 0, JERK_EINTERNAL, "no common segment length");
    for (size_t gi = 0; gi < p.groups.size(); ++gi) {
      Cand bc{JERK_PATH_FFT_FP32, best_seg, 16, best_ept};
      double bt = -1.0;
      for (auto& r : per_group[gi])
        if (r.first.path == JERK_PATH_FFT_FP32 && r.first.seg == best_seg && r.first.ept == best_ept &&
            (bt < 0 || r.second < bt)) {
          bt = r.second;
          bc = r.first;
        }
      p.groups[gi].path = JERK_PATH_FFT_FP32;
      p.groups[gi].seg_len = bc.seg;
      p.groups[gi].tpb = bc.tpb;
      p.groups[gi].ept = bc.ept;
    }
  } else {
    for (size_t gi = 0; gi < p.groups.size(); ++gi) {
      const auto& res = per_group[gi];
      if (res.empty()) continue;
      auto best = std::min_element(res.begin(), res.end(), [](auto& a, auto& b) { return a.second < b.second; });
      Group& g = p.groups[gi];
      g.path = best->first.path;
      if (best->first.path == JERK_PATH_FFT_FP32) {
        g.seg_len = best->first.seg;
        g.tpb = best->first.tpb;
        g.ept = best->first.ept;
      }
    }
  }
  plan_layout(p);
}

}  // namespace jerk

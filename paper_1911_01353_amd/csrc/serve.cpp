// Serving: continuous batching of search requests on one GPU.
//
// A scheduler thread owns the device work. Requests wait in a bounded queue,
// are admitted while their arena footprint (template bank if not cached,
// per-template peak keys and peaks) fits, and are cut into work units (a
// width group's member range over all segments). Each launch slot (its own
// stream) takes units round-robin from every admitted request up to a tile
// budget: FFT units run in one flat launch over a job table, MFMA units
// as direct launches. So requests that arrive while others run share the
// next launches with them instead of waiting behind them. A request's result
// is the per-template maximum over its tiles (an atomicMax of order-free
// keys), identical whatever else ran beside it.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <thread>
#include <vector>

#include "jerk_internal.h"

namespace jerk {
namespace {

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
 public:
  explicit Arena(size_t size = 0) : size_(size) {
    if (size_) free_[0] = size_;
  }
  bool alloc(size_t n, size_t* off) {
    n = align_up(std::max<size_t>(n, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(std::max<size_t>(n, 1));
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct BankEntry {
  std::string key;
  Plan plan;
  size_t off = 0, bytes = 0;
  int refs = 0;
  uint64_t last_use = 0;
  hipEvent_t ready = nullptr;
  bool failed = false;
};

struct Unit {
  int32_t group, m_begin, m_end;
  int64_t tiles;
};

struct Req {
  uint64_t ticket = 0;
  jerk_request r{};
  int state = 0;  // 0 queued, 1 active, 2 done
  BankEntry* bank = nullptr;
  size_t mem_off = 0, mem_bytes = 0;  // keys [T] uint64 then peaks [T] jerk_peak
  hipEvent_t ready = nullptr;         // bank built and keys cleared
  std::vector<Unit> units;
  size_t next_unit = 0;
  int outstanding = 0;
  bool failed = false;
  int32_t fail_status = JERK_OK;
  jerk_result res{};
  std::vector<jerk_peak> peaks;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* pinned = nullptr;   // staged job table
  size_t table_off = 0;     // arena offset of the device job table
  bool busy = false;
  bool inject_fail = false;
  std::vector<std::pair<Req*, int>> reqs;
};

constexpr int32_t kMaxJobsPerLaunch = 512;
constexpr size_t kTableBytes = 256 + sizeof(FftJob) * kMaxJobsPerLaunch;

std::string bank_key(const jerk_request& r, int32_t seg) {
  std::ostringstream o;
  o.precision(17);
  o << r.zmax << '/' << r.wmax << '/' << r.dz << '/' << r.dw << '/' << r.path << '/' << seg;
  return o.str();
}

}  // namespace
}  // namespace jerk

struct jerk_server {
  jerk_serve_desc d{};
  char* arena = nullptr;
  jerk::Arena alloc;
  bool dry = false;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_done, cv_sched;
  std::deque<jerk::Req*> queue;
  std::vector<jerk::Req*> active;
  std::map<uint64_t, std::unique_ptr<jerk::Req>> all;
  std::map<std::string, std::unique_ptr<jerk::BankEntry>> banks;
  std::vector<jerk::Slot> slots;
  hipStream_t build_stream = nullptr;
  hipStream_t fin_stream = nullptr;
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1, use_clock = 0;
  std::chrono::steady_clock::time_point t0;

  int64_t fail_launch_at = 0, fail_build_at = 0, launch_count = 0, build_count = 0;
  int64_t fail_queries = 0;  // completion queries still to fail (test hook)
  bool paused = false;  // admission held (test hook)
  jerk_serve_stats st{};
  size_t rr = 0;  // round-robin start

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace jerk {
namespace {

bool event_done(jerk_server& s, hipEvent_t e) {
  if (s.dry || e == nullptr) return true;
  const hipError_t r = hipEventQuery(e);
  if (r == hipSuccess) return true;
  if (r == hipErrorNotReady) return false;
  throw Error(JERK_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(r));
}

// Completion of a launch slot; the test hook reports a device error for the next queries.
bool slot_done(jerk_server& s, const Slot& sl) {
  if (s.fail_queries > 0) {
    s.fail_queries--;
    throw Error(JERK_EHIP, "hipEventQuery: injected device error");
  }
  return event_done(s, sl.done);
}

void plan_for(const jerk_server& s, const jerk_request& r, Plan& p) {
  jerk_plan_desc d{};
  d.nbins = r.nbins;
  d.zmax = r.zmax;
  d.wmax = r.wmax;
  d.dz = r.dz;
  d.dw = r.dw;
  d.numbetween = 2;
  d.margin_bins = 16;
  d.path = r.path;
  d.seg_len = s.d.seg_len;
  plan_build(p, d);
}

size_t req_mem_bytes(int32_t T) { return align_up((size_t)T * 8) + align_up((size_t)T * sizeof(jerk_peak)); }

void release_bank(jerk_server& s, BankEntry* b) {
  if (!b) return;
  b->refs--;
  if (b->failed && b->refs == 0) {  // a failed build is not kept: the next request rebuilds
    if (!s.dry && b->ready) (void)hipEventDestroy(b->ready);
    s.alloc.release(b->off, b->bytes);
    s.banks.erase(b->key);
  }
}

// Evicts least recently used banks nobody references until `need` bytes fit; true if they do.
bool make_room(jerk_server& s, size_t need, size_t* off) {
  for (;;) {
    if (s.alloc.alloc(need, off)) return true;
    BankEntry* victim = nullptr;
    for (auto& kv : s.banks)
      if (kv.second->refs == 0 && (!victim || kv.second->last_use < victim->last_use)) victim = kv.second.get();
    if (!victim) return false;
    if (!s.dry && victim->ready) {
      (void)hipEventSynchronize(victim->ready);
      (void)hipEventDestroy(victim->ready);
    }
    s.alloc.release(victim->off, victim->bytes);
    s.st.bank_evictions++;
    s.banks.erase(victim->key);
  }
}

void finish(jerk_server& s, Req* q) {
  q->state = 2;
  q->res.t_done = s.now();
  if (q->failed) {
    q->res.status = q->fail_status;
    s.st.failed++;
  } else {
    q->res.status = JERK_OK;
    s.st.completed++;
  }
  if (q->mem_bytes) s.alloc.release(q->mem_off, q->mem_bytes);
  q->mem_bytes = 0;
  release_bank(s, q->bank);
  q->bank = nullptr;
  if (!s.dry && q->ready) (void)hipEventDestroy(q->ready);
  q->ready = nullptr;
  s.cv_done.notify_all();
}

// All units of q have completed: reduce its keys to peaks and fill the result.
void finalize(jerk_server& s, Req* q) {
  const int32_t T = q->res.n_templates;
  q->peaks.assign((size_t)T, jerk_peak{0.f, 0xFFFFFFFFu});
  if (!q->failed && !s.dry) {
    uint64_t* keys = reinterpret_cast<uint64_t*>(s.arena + q->mem_off);
    jerk_peak* dpk = reinterpret_cast<jerk_peak*>(s.arena + q->mem_off + align_up((size_t)T * 8));
    peaks_reduce(keys, T, 1, 1, dpk, s.fin_stream);
    JERK_HIP_CHECK(hipMemcpyAsync(q->peaks.data(), dpk, sizeof(jerk_peak) * T, hipMemcpyDeviceToHost, s.fin_stream));
    JERK_HIP_CHECK(hipStreamSynchronize(s.fin_stream));
  }
  float best = -1.f;
  for (int32_t t = 0; t < T; ++t)
    if (q->peaks[t].power > best) {
      best = q->peaks[t].power;
      q->res.best_power = best;
      q->res.best_t = t;
      q->res.best_p = q->peaks[t].p;
    }
  if (q->r.peaks) std::memcpy(q->r.peaks, q->peaks.data(), sizeof(jerk_peak) * T);
  if (q->r.top && !q->failed) {
    // global top-k over the row peaks: descending power, ties to the lower template
    std::vector<int32_t> idx((size_t)T);
    for (int32_t t = 0; t < T; ++t) idx[t] = t;
    const int32_t k = std::min(q->r.top_capacity, T);
    auto before = [&](int32_t a, int32_t b) {
      return q->peaks[a].power > q->peaks[b].power || (q->peaks[a].power == q->peaks[b].power && a < b);
    };
    std::partial_sort(idx.begin(), idx.begin() + k, idx.end(), before);
    for (int32_t i = 0; i < k; ++i) q->r.top[i] = jerk_top{idx[i], q->peaks[idx[i]].p, q->peaks[idx[i]].power, 0};
    q->res.top_count = k;
  }
  finish(s, q);
}

// Builds the unit list of an admitted request (sizes aim at ~target tiles per unit).
void make_units(jerk_server& s, Req* q, int64_t target) {
  const Plan& p = q->bank->plan;
  for (int32_t gi = 0; gi < (int32_t)p.groups.size(); ++gi) {
    const Group& g = p.groups[gi];
    const int32_t n = (int32_t)g.members.size();
    if (g.path == JERK_PATH_FFT_FP32) {
      const int64_t U = g.seg_len - g.taps + 1;
      const int64_t n_seg = (q->r.nbins + U - 1) / U;
      int32_t blocks = (int32_t)std::max<int64_t>(1, target / n_seg);
      const int32_t step = blocks * g.tpb;
      for (int32_t m = 0; m < n; m += step) {
        const int32_t e = std::min(n, m + step);
        q->units.push_back({gi, m, e, n_seg * ((e - m + g.tpb - 1) / g.tpb)});
      }
    } else {
      // MFMA units: 32 templates (4 row blocks); tile estimate = row blocks x 64-output windows / 8
      const int64_t n_win = (q->r.nbins + 63) / 64;
      const int32_t step = 32;
      for (int32_t m = 0; m < n; m += step) {
        const int32_t e = std::min(n, m + step);
        q->units.push_back({gi, m, e, ((e - m + 7) / 8) * std::max<int64_t>(1, n_win / 8)});
      }
    }
  }
}

// Admits the queue head if its memory fits; returns false when it has to wait.
bool try_admit(jerk_server& s, Req* q) {
  const int32_t seg = s.d.seg_len;
  const std::string key = bank_key(q->r, seg);
  BankEntry* b = nullptr;
  auto it = s.banks.find(key);
  if (it != s.banks.end()) b = it->second.get();
  std::unique_ptr<BankEntry> fresh;
  if (!b) {
    fresh.reset(new BankEntry());
    fresh->key = key;
    plan_for(s, q->r, fresh->plan);
    fresh->bytes = fresh->plan.bank_bytes;
  }
  const int32_t T = b ? b->plan.T : fresh->plan.T;
  size_t mem_off = 0;
  if (b) b->refs++;  // protect from eviction while making room
  const bool mem_ok = make_room(s, req_mem_bytes(T), &mem_off);
  if (!mem_ok) {
    if (b) b->refs--;
    return false;
  }
  if (!b) {
    size_t boff = 0;
    if (!make_room(s, fresh->bytes, &boff)) {
      s.alloc.release(mem_off, req_mem_bytes(T));
      return false;
    }
    fresh->off = boff;
    fresh->refs = 1;
    s.build_count++;
    s.st.bank_builds++;
    const bool inject = s.fail_build_at > 0 && s.build_count == s.fail_build_at;
    if (inject) {
      fresh->failed = true;
    } else if (!s.dry) {
      // a device error here fails this request (below), not the admission loop
      try {
        bank_build(fresh->plan, s.arena + boff, s.build_stream);
        JERK_HIP_CHECK(hipEventCreateWithFlags(&fresh->ready, hipEventDisableTiming));
        JERK_HIP_CHECK(hipEventRecord(fresh->ready, s.build_stream));
      } catch (const Error&) {
        fresh->failed = true;
      }
    }
    b = fresh.get();
    s.banks.emplace(key, std::move(fresh));
  }
  b->last_use = ++s.use_clock;
  q->bank = b;
  q->mem_off = mem_off;
  q->mem_bytes = req_mem_bytes(T);
  q->res.n_templates = T;
  q->res.points = (uint64_t)T * 2 * (uint64_t)q->r.nbins;
  q->res.t_admit = s.now();
  if (b->failed) {
    q->failed = true;
    q->fail_status = JERK_EHIP;
  }
  if (!s.dry && !q->failed) {
    try {
      JERK_HIP_CHECK(hipMemsetAsync(s.arena + mem_off, 0, (size_t)T * 8, s.build_stream));
      JERK_HIP_CHECK(hipEventCreateWithFlags(&q->ready, hipEventDisableTiming));
      JERK_HIP_CHECK(hipEventRecord(q->ready, s.build_stream));
    } catch (const Error& e) {
      q->failed = true;
      q->fail_status = e.status;
    }
  }
  const int64_t target = std::max<int64_t>(256, s.d.tiles_per_launch / std::max(1, s.d.max_active));
  if (!q->failed) make_units(s, q, target);
  q->state = 1;
  return true;
}

// Fills one free slot with units from the active requests; returns whether it launched.
bool dispatch(jerk_server& s, Slot& sl) {
  // A request can take a slot once its template bank is built (a long build must not hold
  // slots). Its keys are cleared on the build stream; the launch stream waits for that on the
  // device (below), so requests admitted together start together in the next launches.
  std::vector<Req*> ready;
  for (Req* q : s.active)
    if (!q->failed && q->next_unit < q->units.size() && event_done(s, q->bank->ready)) ready.push_back(q);
  if (ready.empty()) return false;
  const int64_t budget = s.d.tiles_per_launch;
  std::vector<std::pair<FftJob, std::pair<int32_t, int32_t>>> jobs;  // job, (segment length, elements/thread)
  std::vector<std::pair<Req*, Unit>> gemm;
  std::vector<std::pair<Req*, int>> taken;
  int64_t tiles = 0;
  // round-robin: one unit per request per round until the budget is used
  const size_t start = s.rr++ % ready.size();
  bool any = true;
  while (any && tiles < budget && (int32_t)jobs.size() < kMaxJobsPerLaunch) {
    any = false;
    for (size_t k = 0; k < ready.size() && tiles < budget && (int32_t)jobs.size() < kMaxJobsPerLaunch; ++k) {
      Req* q = ready[(start + k) % ready.size()];
      if (q->next_unit >= q->units.size()) continue;
      const Unit u = q->units[q->next_unit++];
      any = true;
      tiles += u.tiles;
      auto tk = std::find_if(taken.begin(), taken.end(), [&](auto& e) { return e.first == q; });
      if (tk == taken.end()) taken.push_back({q, 1});
      else tk->second++;
      const Plan& p = q->bank->plan;
      const Group& g = p.groups[u.group];
      if (g.path == JERK_PATH_FFT_FP32) {
        const char* bank = s.arena + q->bank->off;
        FftJob j{};
        j.spec = static_cast<const float2*>(q->r.spec);
        j.nbins = q->r.nbins;
        j.bank_fft = reinterpret_cast<const float2*>(bank + g.off_fft);
        j.members = reinterpret_cast<const int32_t*>(bank + p.off_members) + g.first_member;
        j.m_begin = u.m_begin;
        j.m_end = u.m_end;
        j.t_begin = 0;
        j.taps = g.taps;
        j.tpb = g.tpb;
        j.plane = q->r.plane;
        j.ld = q->r.ld;
        j.row_max = reinterpret_cast<uint64_t*>(s.arena + q->mem_off);
        j.rmax_ld = 0;
        jobs.push_back({j, {g.seg_len, g.ept}});
      } else {
        gemm.push_back({q, u});
      }
    }
  }
  if (taken.empty()) return false;
  s.launch_count++;
  s.st.launches++;
  sl.reqs = taken;
  sl.busy = true;
  sl.inject_fail = s.fail_launch_at > 0 && s.launch_count == s.fail_launch_at;
  const double t = s.now();
  for (auto& e : taken)
    if (e.first->res.t_first_launch == 0.0) e.first->res.t_first_launch = t;
  for (auto& e : taken) e.first->outstanding += e.second;
  if (taken.size() >= 2) s.st.shared_launches++;
  int32_t in_flight = 0;
  for (Req* q : s.active) in_flight += q->outstanding > 0;
  s.st.max_in_flight = std::max(s.st.max_in_flight, in_flight);
  if (s.dry || sl.inject_fail) return true;

  for (auto& e : taken) JERK_HIP_CHECK(hipStreamWaitEvent(sl.stream, e.first->ready, 0));
  if (!jobs.empty()) {
    // one launch per segment length present (normally one)
    std::map<std::pair<int32_t, int32_t>, std::vector<FftJob>> by_seg;
    std::map<int32_t, const float2*> tw_of;
    for (auto& e : jobs) by_seg[e.second].push_back(e.first);
    for (auto& e : taken) {
      const Plan& p = e.first->bank->plan;
      for (auto& kv : by_seg)
        tw_of[kv.first.first] =
            reinterpret_cast<const float2*>(s.arena + e.first->bank->off + p.off_tw[tw_slot(kv.first.first)]);
    }
    char* pinned = static_cast<char*>(sl.pinned);
    size_t poff = 0;
    char* dtab = s.arena + sl.table_off;
    for (auto& kv : by_seg) {
      std::vector<FftJob>& js = kv.second;
      int64_t total = 0;
      const int32_t seg = kv.first.first, ept = kv.first.second;
      for (FftJob& j : js) {
        j.tile_begin = total;
        total += fft_job_tiles(j, seg);
      }
      BatchHeader h{};
      h.total_tiles = total;
      h.n_jobs = (int32_t)js.size();
      const size_t bytes = 256 + js.size() * sizeof(FftJob);
      std::memset(pinned + poff, 0, 256);
      std::memcpy(pinned + poff, &h, sizeof(h));
      std::memcpy(pinned + poff + 256, js.data(), js.size() * sizeof(FftJob));
      JERK_HIP_CHECK(hipMemcpyAsync(dtab + poff, pinned + poff, bytes, hipMemcpyHostToDevice, sl.stream));
      // one flat launch over the units of every request taken (a workgroup per tile)
      fft_multi_launch(reinterpret_cast<const FftJob*>(dtab + poff + 256), reinterpret_cast<BatchHeader*>(dtab + poff),
                       total, seg, ept, true, tw_of[seg], sl.stream);
      poff += align_up(bytes);
    }
  }
  for (auto& e : gemm) {
    Req* q = e.first;
    const Unit& u = e.second;
    const Plan& p = q->bank->plan;
    const Group& g = p.groups[u.group];
    const char* bank = s.arena + q->bank->off;
    GemmArgs a{};
    a.spec = static_cast<const float2*>(q->r.spec);
    a.nbins = q->r.nbins;
    a.bank_gemm = bank + g.off_gemm;
    a.members = reinterpret_cast<const int32_t*>(bank + p.off_members) + g.first_member;
    a.m_begin = u.m_begin;
    a.m_end = u.m_end;
    a.t_begin = 0;
    a.t_end = p.T;
    a.plane = q->r.plane;
    a.ld = q->r.ld;
    a.taps = g.taps;
    a.path = g.path;
    a.row_max = reinterpret_cast<uint64_t*>(s.arena + q->mem_off);
    gemm_correlate_launch(a, sl.stream);
  }
  JERK_HIP_CHECK(hipEventRecord(sl.done, sl.stream));
  return true;
}

void scheduler(jerk_server* sp) {
  jerk_server& s = *sp;
  if (!s.dry) (void)hipSetDevice(s.device);
  std::unique_lock<std::mutex> lock(s.mu);
  for (;;) {
    bool progressed = false;
    try {
      // completions
      for (Slot& sl : s.slots) {
        if (sl.busy && slot_done(s, sl)) {
          for (auto& e : sl.reqs) {
            e.first->outstanding -= e.second;
            if (sl.inject_fail && !e.first->failed) {
              e.first->failed = true;
              e.first->fail_status = JERK_EHIP;
            }
          }
          sl.reqs.clear();
          sl.busy = false;
          sl.inject_fail = false;
          progressed = true;
        }
      }
      // finalize
      for (size_t i = 0; i < s.active.size();) {
        Req* q = s.active[i];
        const bool all_launched = q->failed || q->next_unit >= q->units.size();
        if (all_launched && q->outstanding == 0) {
          finalize(s, q);
          s.active.erase(s.active.begin() + i);
          progressed = true;
        } else {
          ++i;
        }
      }
      if (s.stop && s.active.empty()) break;
      // admit
      while (!s.stop && !s.paused && (int32_t)s.active.size() < s.d.max_active && !s.queue.empty()) {
        Req* q = s.queue.front();
        if (!try_admit(s, q)) break;
        s.queue.pop_front();
        s.active.push_back(q);
        progressed = true;
      }
      // dispatch
      for (Slot& sl : s.slots)
        if (!sl.busy && dispatch(s, sl)) progressed = true;
    } catch (const Error& e) {
      // Device error: fail everything active and release every busy slot, so the failed
      // requests reach finalize (host-only for failed requests) and the stop exit stays
      // reachable; the server keeps accepting work.
      for (Req* q : s.active) {
        q->failed = true;
        q->fail_status = e.status;
      }
      for (Slot& sl : s.slots) {
        if (!sl.busy) continue;
        if (!s.dry) (void)hipStreamSynchronize(sl.stream);  // its pinned table is free again
        for (auto& r : sl.reqs) r.first->outstanding -= r.second;
        sl.reqs.clear();
        sl.busy = false;
        sl.inject_fail = false;
      }
      progressed = true;
    }
    s.st.queued = (int32_t)s.queue.size();
    s.st.active = (int32_t)s.active.size();
    s.st.arena_used = s.alloc.used();
    if (!progressed) {
      bool inflight = false;
      for (Slot& sl : s.slots) inflight = inflight || sl.busy;
      bool building = false;
      for (Req* q : s.active) building = building || q->next_unit < q->units.size();
      if (inflight || building) {
        lock.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lock.lock();
      } else {
        s.cv_sched.wait_for(lock, std::chrono::milliseconds(50));
      }
    }
  }
}

void validate_request(const jerk_request& r) {
  require(r.spec != nullptr && r.nbins >= 1, JERK_EINVAL, "request spectrum must be set and nbins >= 1");
  require(2 * r.nbins <= 0xFFFFFFFFll, JERK_EINVAL, "nbins too large for 32-bit plane indices");
  require(r.path == JERK_PATH_FFT_FP32 || r.path == JERK_PATH_GEMM_SPLIT_BF16, JERK_EINVAL,
          "request path must be FFT_FP32 or GEMM_SPLIT_BF16");
  require(!r.plane || (r.ld >= 2 * r.nbins && r.ld % 2 == 0), JERK_EINVAL, "plane ld must be even and >= 2 nbins");
  require(reinterpret_cast<uintptr_t>(r.spec) % 8 == 0 && reinterpret_cast<uintptr_t>(r.plane) % 8 == 0, JERK_EINVAL,
          "request buffers must be 8-byte aligned");
  require(r.top_capacity >= 0 && (r.top != nullptr) == (r.top_capacity > 0), JERK_EINVAL,
          "top must be set exactly when top_capacity > 0");
}

}  // namespace

void serve_create(const jerk_serve_desc& d, void* d_arena, size_t arena_bytes, jerk_server** out) {
  require(d.max_active >= 1 && d.queue_capacity >= 1, JERK_EINVAL, "max_active and queue_capacity must be >= 1");
  require(d.tiles_per_launch >= 0, JERK_EINVAL, "tiles_per_launch must be >= 0");
  require(d.seg_len == 0 || seg_len_supported(d.seg_len), JERK_EINVAL, "seg_len must be 0 or 512..4096");
  require(d.slots >= 0 && d.slots <= 8, JERK_EINVAL, "slots must be in [0, 8]");
  require((d.flags & ~JERK_SERVE_DRYRUN) == 0, JERK_EINVAL, "unknown flags");
  require(d_arena != nullptr && reinterpret_cast<uintptr_t>(d_arena) % 256 == 0, JERK_EINVAL,
          "arena must be set and 256-byte aligned");
  std::unique_ptr<jerk_server> s(new jerk_server());
  s->d = d;
  if (s->d.slots == 0) s->d.slots = 3;
  if (s->d.tiles_per_launch == 0) s->d.tiles_per_launch = 1 << 16;
  s->arena = static_cast<char*>(d_arena);
  s->dry = (d.flags & JERK_SERVE_DRYRUN) != 0;
  s->t0 = std::chrono::steady_clock::now();
  const size_t tables = (size_t)s->d.slots * align_up(kTableBytes) * 2;
  require(arena_bytes > tables + (1 << 20), JERK_ENOMEM, "arena too small for the launch tables");
  s->alloc = Arena(arena_bytes);
  s->st.arena_bytes = arena_bytes;
  s->slots.resize(s->d.slots);
  try {
    if (!s->dry) {
      JERK_HIP_CHECK(hipGetDevice(&s->device));
      JERK_HIP_CHECK(hipStreamCreateWithFlags(&s->build_stream, hipStreamNonBlocking));
      JERK_HIP_CHECK(hipStreamCreateWithFlags(&s->fin_stream, hipStreamNonBlocking));
    }
    for (Slot& sl : s->slots) {
      bool ok = s->alloc.alloc(align_up(kTableBytes) * 2, &sl.table_off);
      require(ok, JERK_ENOMEM, "arena too small for the launch tables");
      if (!s->dry) {
        JERK_HIP_CHECK(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
        JERK_HIP_CHECK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
        JERK_HIP_CHECK(hipHostMalloc(&sl.pinned, align_up(kTableBytes) * 2, hipHostMallocDefault));
      }
    }
  } catch (...) {
    for (Slot& sl : s->slots) {
      if (sl.pinned) (void)hipHostFree(sl.pinned);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->build_stream) (void)hipStreamDestroy(s->build_stream);
    if (s->fin_stream) (void)hipStreamDestroy(s->fin_stream);
    throw;
  }
  jerk_server* raw = s.release();
  raw->th = std::thread(scheduler, raw);
  *out = raw;
}

void serve_submit(jerk_server& s, const jerk_request& r, uint64_t* ticket) {
  validate_request(r);
  // footprint check against the whole arena (can this request ever run?)
  Plan probe;
  plan_for(s, r, probe);
  require(!r.peaks || r.peaks_capacity >= probe.T, JERK_EINVAL, "peaks_capacity smaller than n_templates");
  const size_t fixed = (size_t)s.d.slots * align_up(kTableBytes) * 2;
  require(fixed + align_up(probe.bank_bytes) + req_mem_bytes(probe.T) <= s.alloc.size(), JERK_ENOMEM,
          "request footprint exceeds the arena");
  std::unique_ptr<Req> q(new Req());
  q->r = r;
  std::lock_guard<std::mutex> lock(s.mu);
  require(!s.stop, JERK_EINVAL, "server is stopping");
  require((int32_t)s.queue.size() < s.d.queue_capacity, JERK_EAGAIN, "queue full");
  q->ticket = s.next_ticket++;
  q->res.t_submit = s.now();
  q->res.n_templates = probe.T;
  *ticket = q->ticket;
  s.queue.push_back(q.get());
  s.all.emplace(q->ticket, std::move(q));
  s.st.submitted++;
  s.cv_sched.notify_all();
}

int32_t serve_poll(jerk_server& s, uint64_t ticket, jerk_result* out, double timeout_s) {
  std::unique_lock<std::mutex> lock(s.mu);
  auto it = s.all.find(ticket);
  require(it != s.all.end(), JERK_EINVAL, "unknown ticket");
  Req* q = it->second.get();
  if (q->state != 2 && timeout_s != 0.0) {
    auto pred = [&] { return q->state == 2; };
    if (timeout_s < 0) s.cv_done.wait(lock, pred);
    else s.cv_done.wait_for(lock, std::chrono::duration<double>(timeout_s), pred);
  }
  if (q->state != 2) return JERK_EPENDING;
  *out = q->res;
  return JERK_OK;
}

void serve_stats(jerk_server& s, jerk_serve_stats* out) {
  std::lock_guard<std::mutex> lock(s.mu);
  *out = s.st;
  out->queued = (int32_t)s.queue.size();
  out->active = (int32_t)s.active.size();
  out->arena_used = s.alloc.used();
}

void serve_inject(jerk_server& s, int32_t op, int64_t n) {
  require(op >= 1 && op <= 4, JERK_EINVAL,
          "op must be 1 (launch), 2 (bank build), 3 (hold admission) or 4 (completion query errors)");
  require(n >= 0, JERK_EINVAL, "n must be >= 0");
  std::lock_guard<std::mutex> lock(s.mu);
  if (op == 1) s.fail_launch_at = n ? s.launch_count + n : 0;
  else if (op == 2) s.fail_build_at = n ? s.build_count + n : 0;
  else if (op == 3) s.paused = n != 0;
  else s.fail_queries = n;
  s.cv_sched.notify_all();
}

void serve_destroy(jerk_server* s) {
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
    for (Req* q : s->queue) {
      q->state = 2;
      q->res.status = JERK_ECANCELED;
      q->res.t_done = s->now();
    }
    s->queue.clear();
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  if (!s->dry) {
    for (auto& kv : s->banks)
      if (kv.second->ready) {
        (void)hipEventSynchronize(kv.second->ready);
        (void)hipEventDestroy(kv.second->ready);
      }
    for (Slot& sl : s->slots) {
      if (sl.stream) (void)hipStreamSynchronize(sl.stream);
      if (sl.pinned) (void)hipHostFree(sl.pinned);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->build_stream) {
      (void)hipStreamSynchronize(s->build_stream);
      (void)hipStreamDestroy(s->build_stream);
    }
    if (s->fin_stream) (void)hipStreamDestroy(s->fin_stream);
    for (auto& kv : s->banks)
      if (kv.second->plan.pinned_members) (void)hipHostFree(kv.second->plan.pinned_members);
  }
  delete s;
}

}  // namespace jerk

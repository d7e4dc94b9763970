// Batched search: many spectra of any lengths in one persistent kernel launch,
// optionally captured in a hipGraph and replayed. The host builds a job table
// (one job per spectrum and width group), stages it through pinned memory
// into the caller's workspace and launches the persistent kernel, whose
// workgroups take tiles from a device counter.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "jerk_internal.h"

namespace jerk {

struct BatchCtx {
  std::mutex mu;
  int device = -1;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t staged = nullptr;  // completes when the last staging copy has been consumed
  hipStream_t stream = nullptr; // capture / replay stream
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* graph_ws = nullptr;
  const void* graph_tw = nullptr;
  int32_t graph_seg = 0, graph_ept = 0;
  int64_t graph_grid = 0;
  bool graph_keys = false, graph_flat = false;
  int32_t grid_cache_seg = 0, grid_cache_ept = 0, grid_cache = 0;
};

void batch_ctx_free(BatchCtx* c) {
  if (!c) return;
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->staged) (void)hipEventDestroy(c->staged);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

namespace {

constexpr size_t kHeaderBytes = 256;

size_t jobs_capacity_bytes(const Plan& p, int32_t count) {
  return kHeaderBytes + align_up((size_t)count * p.groups.size() * sizeof(FftJob));
}

// The one (segment length, elements per thread) FFT variant of all groups.
std::pair<int32_t, int32_t> uniform_variant(const Plan& p) {
  int32_t s = 0, e = 0;
  for (const Group& g : p.groups) {
    require(g.path == JERK_PATH_FFT_FP32, JERK_EINVAL,
            "batched search runs the FFT path: every width group must use JERK_PATH_FFT_FP32");
    require(s == 0 || (s == g.seg_len && e == g.ept), JERK_EINVAL,
            "batched search needs one FFT segment length and kernel variant for all width groups "
            "(plan seg_len or the autotuner's uniform mode)");
    s = g.seg_len;
    e = g.ept;
  }
  return {s, e};
}

}  // namespace

size_t batch_workspace_bytes(const Plan& p, int32_t count) { return jobs_capacity_bytes(p, count); }

int64_t batch_keys_per_row(const Plan& p, int64_t nbins) {
  int64_t most = 0;
  for (const Group& g : p.groups) {
    const int64_t U = g.seg_len - g.taps + 1;
    most = std::max(most, (nbins + U - 1) / U);
  }
  return most;
}

void batch_search(Plan& p, const void* d_bank, const jerk_batch_item* items, int32_t count, int32_t t_begin,
                  int32_t t_end, void* d_ws, size_t ws_bytes, uint32_t flags, hipStream_t stream) {
  require(d_bank != nullptr, JERK_EINVAL, "bank must not be NULL");
  require(count >= 0 && (count == 0 || items != nullptr), JERK_EINVAL, "items must not be NULL");
  require(0 <= t_begin && t_begin <= t_end && t_end <= p.T, JERK_EINVAL, "template range outside [0, n_templates]");
  require((flags & ~(JERK_BATCH_GRAPH | JERK_BATCH_FLAT | JERK_BATCH_PERSISTENT)) == 0, JERK_EINVAL, "unknown flags");
  require((flags & JERK_BATCH_FLAT) == 0 || (flags & JERK_BATCH_PERSISTENT) == 0, JERK_EINVAL,
          "JERK_BATCH_FLAT and JERK_BATCH_PERSISTENT exclude each other");
  const bool flat = (flags & JERK_BATCH_PERSISTENT) == 0;
  const auto var = uniform_variant(p);
  const int32_t seg = var.first, ept = var.second;
  const size_t need = jobs_capacity_bytes(p, count);
  require(d_ws != nullptr && ws_bytes >= need, JERK_ENOMEM, "workspace smaller than jerk_batch_workspace_bytes");
  require(reinterpret_cast<uintptr_t>(d_ws) % 256 == 0, JERK_EINVAL, "workspace must be 256-byte aligned");
  for (int32_t i = 0; i < count; ++i) {
    const jerk_batch_item& it = items[i];
    require(it.spec != nullptr && it.nbins >= 1, JERK_EINVAL, "item spectrum must be set and nbins >= 1");
    require(it.plane != nullptr || it.peaks != nullptr, JERK_EINVAL, "item needs a plane or a peak buffer");
    require(!it.plane || (it.ld >= 2 * it.nbins && it.ld % 2 == 0), JERK_EINVAL, "item ld must be even and >= 2 nbins");
    require(!it.peaks || it.keys_ld >= batch_keys_per_row(p, it.nbins), JERK_EINVAL,
            "item keys_ld smaller than jerk_batch_keys_per_row");
    require(reinterpret_cast<uintptr_t>(it.spec) % 8 == 0 && reinterpret_cast<uintptr_t>(it.plane) % 8 == 0,
            JERK_EINVAL, "item buffers must be 8-byte aligned");
  }

  bool keys = false;
  for (int32_t i = 0; i < count; ++i) {
    require(i == 0 || (items[i].peaks != nullptr) == keys, JERK_EINVAL,
            "either every item of a batch has a peak buffer or none has");
    keys = items[i].peaks != nullptr;
  }
  const char* bank = static_cast<const char*>(d_bank);
  const int32_t* members = reinterpret_cast<const int32_t*>(bank + p.off_members);
  std::vector<FftJob> jobs;
  jobs.reserve((size_t)count * p.groups.size());
  int64_t total = 0;
  for (int32_t i = 0; i < count; ++i) {
    const jerk_batch_item& it = items[i];
    for (const Group& g : p.groups) {
      const int32_t lo = (int32_t)(std::lower_bound(g.members.begin(), g.members.end(), t_begin) - g.members.begin());
      const int32_t hi = (int32_t)(std::lower_bound(g.members.begin(), g.members.end(), t_end) - g.members.begin());
      if (lo >= hi) continue;
      FftJob j{};
      j.spec = static_cast<const float2*>(it.spec);
      j.nbins = it.nbins;
      j.bank_fft = reinterpret_cast<const float2*>(bank + g.off_fft);
      j.members = members + g.first_member;
      j.m_begin = lo;
      j.m_end = hi;
      j.t_begin = t_begin;
      j.taps = g.taps;
      j.tpb = g.tpb;
      j.plane = it.plane;
      j.ld = it.ld;
      j.row_max = it.peaks;
      j.rmax_ld = it.keys_ld;
      j.tile_begin = total;
      total += fft_job_tiles(j, seg);
      jobs.push_back(j);
    }
  }
  if (jobs.empty()) return;

  if (!p.batch) p.batch = new BatchCtx();
  BatchCtx& c = *p.batch;
  std::lock_guard<std::mutex> lock(c.mu);
  int dev = 0;
  JERK_HIP_CHECK(hipGetDevice(&dev));
  if (c.device < 0) {
    c.device = dev;
    JERK_HIP_CHECK(hipEventCreateWithFlags(&c.staged, hipEventDisableTiming));
    JERK_HIP_CHECK(hipEventCreateWithFlags(&c.ev_in, hipEventDisableTiming));
    JERK_HIP_CHECK(hipEventCreateWithFlags(&c.ev_out, hipEventDisableTiming));
    JERK_HIP_CHECK(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
  }
  require(c.device == dev, JERK_EINVAL, "a plan's batched launches must stay on one device");
  if (c.grid_cache_seg != seg || c.grid_cache_ept != ept) {
    c.grid_cache = fft_persistent_grid(seg, ept);
    c.grid_cache_seg = seg;
    c.grid_cache_ept = ept;
  }
  const int32_t grid = (int32_t)std::min<int64_t>(c.grid_cache, total);

  // Stage header + jobs. The staging buffer is reused: wait for the previous copy.
  const size_t bytes = kHeaderBytes + jobs.size() * sizeof(FftJob);
  JERK_HIP_CHECK(hipEventSynchronize(c.staged));
  if (c.pinned_bytes < bytes) {
    if (c.pinned) JERK_HIP_CHECK(hipHostFree(c.pinned));
    c.pinned = nullptr;
    c.pinned_bytes = 0;
    JERK_HIP_CHECK(hipHostMalloc(&c.pinned, bytes, hipHostMallocDefault));
    c.pinned_bytes = bytes;
  }
  BatchHeader h{};
  h.total_tiles = total;
  h.counter = 0;
  h.n_jobs = (int32_t)jobs.size();
  std::memset(c.pinned, 0, kHeaderBytes);
  std::memcpy(c.pinned, &h, sizeof(h));
  std::memcpy(static_cast<char*>(c.pinned) + kHeaderBytes, jobs.data(), jobs.size() * sizeof(FftJob));
  char* ws = static_cast<char*>(d_ws);
  BatchHeader* d_hdr = reinterpret_cast<BatchHeader*>(ws);
  const FftJob* d_jobs = reinterpret_cast<const FftJob*>(ws + kHeaderBytes);
  const float2* tw = reinterpret_cast<const float2*>(bank + p.off_tw[tw_slot(seg)]);

  if (!(flags & JERK_BATCH_GRAPH)) {
    JERK_HIP_CHECK(hipMemcpyAsync(ws, c.pinned, bytes, hipMemcpyHostToDevice, stream));
    JERK_HIP_CHECK(hipEventRecord(c.staged, stream));
    if (flat) fft_multi_launch(d_jobs, d_hdr, total, seg, ept, keys, tw, stream);
    else fft_persistent_launch(d_jobs, d_hdr, seg, ept, keys, tw, grid, stream);
    return;
  }
  // Graph path: the graph holds the counter reset and the persistent kernel;
  // its arguments (workspace, twiddles, grid) fix the graph, the job table does not.
  // (persistent: a full-size grid, so one graph serves any tile count; flat: the grid is the tile count)
  const int64_t ggrid = flat ? total : c.grid_cache;
  if (!c.exec || c.graph_ws != d_ws || c.graph_tw != tw || c.graph_seg != seg || c.graph_ept != ept ||
      c.graph_grid != ggrid || c.graph_keys != keys || c.graph_flat != flat) {
    if (c.exec) JERK_HIP_CHECK(hipGraphExecDestroy(c.exec));
    if (c.graph) JERK_HIP_CHECK(hipGraphDestroy(c.graph));
    c.exec = nullptr;
    c.graph = nullptr;
    JERK_HIP_CHECK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
    try {
      if (flat) fft_multi_launch(d_jobs, d_hdr, ggrid, seg, ept, keys, tw, c.stream);
      else fft_persistent_launch(d_jobs, d_hdr, seg, ept, keys, tw, (int32_t)ggrid, c.stream);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(c.stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    JERK_HIP_CHECK(hipStreamEndCapture(c.stream, &c.graph));
    JERK_HIP_CHECK(hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0));
    c.graph_ws = d_ws;
    c.graph_tw = tw;
    c.graph_seg = seg;
    c.graph_ept = ept;
    c.graph_keys = keys;
    c.graph_grid = ggrid;
    c.graph_flat = flat;
  }
  JERK_HIP_CHECK(hipEventRecord(c.ev_in, stream));
  JERK_HIP_CHECK(hipStreamWaitEvent(c.stream, c.ev_in, 0));
  JERK_HIP_CHECK(hipMemcpyAsync(ws, c.pinned, bytes, hipMemcpyHostToDevice, c.stream));
  JERK_HIP_CHECK(hipEventRecord(c.staged, c.stream));
  JERK_HIP_CHECK(hipGraphLaunch(c.exec, c.stream));
  JERK_HIP_CHECK(hipEventRecord(c.ev_out, c.stream));
  JERK_HIP_CHECK(hipStreamWaitEvent(stream, c.ev_out, 0));
}

}  // namespace jerk

// Serving form of libppf.so: continuous batching of chunks from many
// streams of different N and T onto the GPU.
//
// Producers push chunks from any thread into a lock-free submission queue.
// One scheduler thread per server
//   1. moves new submissions into per-stream FIFOs and admits waiting
//      streams as the state budget allows,
//   2. as soon as an in-flight slot is free, forms a batch: for every
//      admitted stream its ready chunks in order (a later chunk of a stream
//      joins only when the one before it has at least T-1 spectra, so that
//      its history is a contiguous tail of that chunk), split into tiles,
//   3. writes the batch's descriptor table into the slot's pinned buffer and
//      replays the slot's captured graph: the descriptor copy, then one
//      branch per plan class (fused kernel, or FIR then FFT through the
//      slot's workspace), and the history-update kernel,
//   4. polls the slots' completion events and stamps chunk latencies.
// Batches run in launch order on one HIP stream; the class branches of a
// batch run concurrently. A stream's history lives in device memory (two
// buffers; each batch that touches the stream reads one and writes the
// other).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "../../include/ppf.h"
#include "ppf_internal.h"

namespace {

#ifndef PPF_SERVER_FIR_TILE
#define PPF_SERVER_FIR_TILE 32
#endif
// Batches of different slots on their own streams (concurrent on the GPU);
// a stream then joins a batch only when none of its chunks is in flight.
#ifndef PPF_SERVER_CONCURRENT_SLOTS
#define PPF_SERVER_CONCURRENT_SLOTS 0
#endif
// Fused/FFT tile length per class chosen to spread each class over about
// this many tiles (0: fixed tiles of about 32K samples).
#ifndef PPF_SERVER_TARGET_TILES
#define PPF_SERVER_TARGET_TILES 256
#endif
constexpr int kMaxClasses = 8;
constexpr int kMaxTiles = 6144;       // per batch, all classes
constexpr int kTargetTiles = PPF_SERVER_TARGET_TILES;   // tiles per plan class and batch
constexpr int kMaxHist = 512;         // history entries per batch
constexpr int kMaxSlots = 4;
constexpr size_t kSlotWorkspace = 512ull << 20;  // two-pass presums per batch
constexpr long long kMaxChunkSpectra = 1ll << 31;

long long now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// descriptor area (identical layout on host and device)
struct DescArea {
  ppf::DescClass fused[kMaxClasses];
  ppf::DescClass fir[kMaxClasses];
  ppf::DescClass fft[kMaxClasses];
  int nhist;
  int pad_[3];
  ppf::HistDesc hist[kMaxHist];
  ppf::TileDesc tiles[kMaxTiles];   // last: a batch uploads only the tiles it uses
};

struct PendingChunk {
  ppf_chunk c;
  long long arrival_ns;
  bool last;          // the last piece of a pushed chunk: its completion reports the tag
};

}  // namespace

namespace ppf {

// Per-stream state of a server stream, shared by the server's table and
// the stream handle (whichever lets go last frees it).
struct SrvStream {
  int id = -1;
  ppf_plan_t plan = nullptr;
  int cls = -1;
  int N = 0;
  long long max_piece = 1;          // spectra per queued piece (the class limit)
  void* hist[2] = {nullptr, nullptr};
  int cur = 0;                      // scheduler
  long long hist_samples = 0;
  size_t state_bytes = 0;
  std::atomic<bool> admitted{false};
  std::atomic<bool> closing{false};
  bool dropped = false;             // closed before admission: its chunks are dropped (mu)
  std::deque<PendingChunk> queue;   // scheduler-owned FIFO (mu)
  std::atomic<long long> outstanding{0};   // pieces submitted, not completed or dropped
  long long inflight = 0;           // in a launched batch, not completed (scheduler)
};

}  // namespace ppf

namespace {

using ppf::SrvStream;

struct DoneChunk {
  unsigned long long tag;
  long long arrival_ns;
  long long bytes;
  long long spectra;
  SrvStream* stream;
  bool last;
};

struct Slot {
  DescArea* host = nullptr;        // pinned
  DescArea* dev = nullptr;
  size_t upload_bytes = 0;         // used prefix of the descriptor area
  hipStream_t stream = nullptr;    // batches of different slots run concurrently
  void* ws = nullptr;
  hipEvent_t done = nullptr;
  hipEvent_t start = nullptr;      // timing: recorded before the graph
  hipGraphExec_t exec = nullptr;
  int graph_classes = -1;          // class count the graph was captured for
  bool busy = false;
  std::vector<DoneChunk> chunks;
};

struct ClassInfo {
  ppf_plan_t plan = nullptr;
  int N = 0, T = 0;
  bool fused = true;
  int tile_spectra = 16;       // fused and FFT-pass tiles (spread over workgroups)
  int fir_tile_spectra = PPF_SERVER_FIR_TILE;   // FIR-pass tiles (channels give the parallelism; long tiles
                               // read the T-1 halo blocks fewer times)
  long long max_piece = 1;     // spectra of the largest piece an empty batch takes
};

// One submission on its way from a producer thread to the scheduler.
struct Submission {
  SrvStream* stream;
  PendingChunk pc;
};

// Bounded multi-producer queue of submissions: the array-based queue of
// D. Vyukov, in which each cell carries a sequence number telling whether
// it is free for the producer that claims its position or full for the
// consumer reading there. Producers never take a lock; the scheduler
// thread is the only consumer.
class SubmitQueue {
 public:
  explicit SubmitQueue(size_t cap_pow2) : cells_(new Cell[cap_pow2]), mask_(cap_pow2 - 1) {
    for (size_t i = 0; i < cap_pow2; ++i) cells_[i].seq.store(i, std::memory_order_relaxed);
  }
  // false when the queue is full
  bool push(const Submission& v) {
    size_t pos = enq_.load(std::memory_order_relaxed);
    for (;;) {
      Cell& c = cells_[pos & mask_];
      const size_t seq = c.seq.load(std::memory_order_acquire);
      const intptr_t dif = (intptr_t)seq - (intptr_t)pos;
      if (dif == 0) {
        if (enq_.compare_exchange_weak(pos, pos + 1, std::memory_order_relaxed)) {
          c.v = v;
          c.seq.store(pos + 1, std::memory_order_seq_cst);
          return true;
        }
      } else if (dif < 0) {
        return false;
      } else {
        pos = enq_.load(std::memory_order_relaxed);
      }
    }
  }
  // consumer only
  bool pop(Submission& v) {
    Cell& c = cells_[deq_ & mask_];
    const size_t seq = c.seq.load(std::memory_order_acquire);
    if ((intptr_t)seq - (intptr_t)(deq_ + 1) < 0) return false;
    v = c.v;
    c.seq.store(deq_ + mask_ + 1, std::memory_order_release);
    ++deq_;
    return true;
  }
  bool empty() const {   // consumer only
    const Cell& c = cells_[deq_ & mask_];
    return (intptr_t)c.seq.load(std::memory_order_seq_cst) - (intptr_t)(deq_ + 1) < 0;
  }

 private:
  struct Cell {
    std::atomic<size_t> seq;
    Submission v;
  };
  std::unique_ptr<Cell[]> cells_;
  const size_t mask_;
  alignas(64) std::atomic<size_t> enq_{0};
  alignas(64) size_t deq_ = 0;
};
constexpr size_t kSubmitQueueCells = 1u << 16;

// Chunk latencies in a log-spaced histogram: bins of 0.4% relative width
// from 0.5 us to beyond 100 s, so percentiles take O(bins) work and memory
// does not grow with the number of chunks.
class LatencyHist {
 public:
  static constexpr double kLo = 0.5;          // us
  static constexpr double kRatio = 1.004;
  static constexpr int kBins = 4800;          // kLo * kRatio^(kBins-1) > 1e8 us
  void add(double us) {
    int b = 0;
    if (us > kLo) b = std::min(kBins - 1, 1 + (int)(std::log(us / kLo) / std::log(kRatio)));
    counts_[b]++;
    n_++;
    sum_ += us;
    if (n_ == 1 || us > max_) max_ = us;
    if (n_ == 1 || us < min_) min_ = us;
  }
  void clear() {
    std::fill(counts_.begin(), counts_.end(), 0);
    n_ = 0;
    sum_ = max_ = min_ = 0;
  }
  long long count() const { return n_; }
  double mean() const { return n_ ? sum_ / n_ : 0.0; }
  double max() const { return max_; }
  // the value of rank p*(n-1): the geometric centre of its bin (0.2% from
  // any value in it), clamped to the observed range
  double pct(double p) const {
    if (n_ == 0) return 0.0;
    const long long rank = (long long)(p * (double)(n_ - 1) + 0.5);
    long long acc = 0;
    int b = 0;
    for (; b < kBins - 1; ++b) {
      acc += counts_[b];
      if (acc > rank) break;
    }
    const double v = b == 0 ? kLo : kLo * std::pow(kRatio, b - 0.5);
    return std::min(max_, std::max(min_, v));
  }

 private:
  std::vector<long long> counts_ = std::vector<long long>(kBins, 0);
  long long n_ = 0;
  double sum_ = 0, max_ = 0, min_ = 0;
};

// completed tags kept for ppf_server_poll; the oldest are dropped beyond this
constexpr size_t kMaxDoneTags = 1u << 22;

thread_local int s_status = PPF_OK;

int sfail(int st, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  s_status = st;
  ppf_internal_set_error(st, msg);
  return st;
}

int sfail_hip(hipError_t e, const char* what) {
  return sfail(e == hipErrorOutOfMemory ? PPF_ERR_NOMEM : PPF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

struct ppf_server_s {
  size_t budget = 0;
  int nslots = 2;
  Slot slots[kMaxSlots];
  int next_slot = 0;               // the slot launched next (launch order = completion order)
  hipStream_t launch = nullptr;
  hipStream_t branch[kMaxClasses] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxClasses] = {};
  hipStream_t hist_branch = nullptr;   // history updates of a batch
  hipEvent_t hist_join = nullptr;

  SubmitQueue subq{kSubmitQueueCells};
  std::atomic<long long> outstanding{0};   // pieces submitted, not completed or dropped
  std::atomic<bool> sleeping{false};       // the scheduler waits on cv
  std::atomic<int> async_error{PPF_OK};
  std::atomic<bool> stop{false};

  std::mutex mu;                   // guards the stream table, classes, admission, scheduling
  std::condition_variable cv;      // wakes the scheduler, signals drains
  size_t used = 0;                 // state bytes of admitted streams + fixed buffers
  std::vector<ClassInfo> classes;
  std::map<int, std::shared_ptr<SrvStream>> streams;
  std::set<ppf_stream_s*> handles; // open handles (orphaned when the server goes)
  std::deque<int> waiting;         // streams waiting for admission, in order
  std::vector<void*> deferred_free;   // history buffers of released streams, freed when idle
  std::vector<SrvStream*> order;   // admitted-stream visiting order of form_batch
  bool order_stale = true;
  size_t rr = 0;                   // rotating start of form_batch's visit
  int next_id = 0;
  long long stat_admitted = 0, stat_rejected = 0, stat_queued = 0;

  std::mutex dmu;                  // guards completions and statistics below
  std::deque<unsigned long long> done_tags;
  long long tags_dropped = 0;
  LatencyHist lat;
  long long stat_chunks = 0, stat_spectra = 0, stat_bytes = 0, stat_batches = 0;
  double stat_gpu_us = 0, stat_form_us = 0, stat_launch_us = 0;
  long long stat_timed = 0;
  long long first_arrival = -1, last_done = -1;

  std::thread worker;
};

namespace {

size_t stream_state_bytes(int N, int T) { return 2ull * (size_t)(T - 1) * N * 8 + 4096; }

// Largest piece of a chunk one batch can hold on its own: the tiles of the
// piece (at the class's longest tiles) and, for two-pass classes, its
// presums in the slot workspace.
long long max_piece_spectra(const ClassInfo& ci) {
  if (ci.fused) return (long long)kMaxTiles * ci.tile_spectra;
  const long long by_ws = (long long)(kSlotWorkspace / ((size_t)ci.N * 8));
  long long s = std::min<long long>(by_ws, (long long)kMaxTiles * ci.tile_spectra);
  auto tiles = [&](long long S) {
    return (S + ci.tile_spectra - 1) / ci.tile_spectra + (S + ci.fir_tile_spectra - 1) / ci.fir_tile_spectra;
  };
  while (s > 1 && tiles(s) > kMaxTiles) s -= std::max<long long>(1, (tiles(s) - kMaxTiles) * ci.fir_tile_spectra / 2);
  return std::max<long long>(1, s);
}

int class_of(ppf_server_s* s, ppf_plan_t plan) {
  for (size_t i = 0; i < s->classes.size(); ++i)
    if (s->classes[i].plan == plan) return (int)i;
  if ((int)s->classes.size() >= kMaxClasses) return -1;
  ClassInfo ci;
  ci.plan = plan;
  long long v = 0;
  ppf_plan_query(plan, PPF_Q_N, &v);
  ci.N = (int)v;
  ppf_plan_query(plan, PPF_Q_TAPS, &v);
  ci.T = (int)v;
  ppf_plan_query(plan, PPF_Q_PATH, &v);
  ci.fused = v == PPF_PATH_FUSED;
  // tiles of about 32K samples, 4..64 spectra (build-time tuning)
#ifndef PPF_SERVER_TILE_SAMPLES
#define PPF_SERVER_TILE_SAMPLES 32768
#endif
#ifndef PPF_SERVER_TILE_MAX
#define PPF_SERVER_TILE_MAX 64
#endif
  int ts = PPF_SERVER_TILE_SAMPLES / ci.N;
  ci.tile_spectra = ts < 4 ? 4 : (ts > PPF_SERVER_TILE_MAX ? PPF_SERVER_TILE_MAX : ts);
  ci.max_piece = max_piece_spectra(ci);
  s->classes.push_back(ci);
  return (int)s->classes.size() - 1;
}

// The work of one batch in slot `sl` after its descriptor upload on
// s->launch: a fork into one branch per plan class and one for the history
// updates, joined back into s->launch.
hipError_t enqueue_batch(ppf_server_s* s, Slot& sl) {
  hipError_t e = hipEventRecord(s->fork, s->launch);
  const int nc = (int)s->classes.size();
  // history updates read only the old history and the chunks: a branch of
  // their own, beside the transforms
  long long max_hist = 1;
  for (const ClassInfo& ci : s->classes) max_hist = std::max<long long>(max_hist, (long long)(ci.T - 1) * ci.N);
  if (e == hipSuccess) e = hipStreamWaitEvent(s->hist_branch, s->fork, 0);
  if (e == hipSuccess) e = ppf::launch_history_desc(&sl.dev->nhist, sl.dev->hist, kMaxHist, max_hist, s->hist_branch);
  if (e == hipSuccess) e = hipEventRecord(s->hist_join, s->hist_branch);
  if (e == hipSuccess) e = hipStreamWaitEvent(s->launch, s->hist_join, 0);
  for (int c = 0; c < nc && e == hipSuccess; ++c) {
    hipStream_t b = s->branch[c];
    e = hipStreamWaitEvent(b, s->fork, 0);
    if (e != hipSuccess) break;
    const ppf::PlanDev pd = ppf_internal_plan_dev(s->classes[c].plan);
    if (s->classes[c].fused) {
      e = ppf::launch_fused_desc(pd, &sl.dev->fused[c], sl.dev->tiles, kMaxTiles, b);
    } else {
      e = ppf::launch_fir_desc(pd, &sl.dev->fir[c], sl.dev->tiles, kMaxTiles, b);
      if (e == hipSuccess) e = ppf::launch_fft_desc(pd, &sl.dev->fft[c], sl.dev->tiles, kMaxTiles, b);
    }
    if (e == hipSuccess) e = hipEventRecord(s->join[c], b);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->launch, s->join[c], 0);
  }
  return e;
}

// Batches replay a captured graph of enqueue_batch (one launch call) unless
// built with PPF_SERVER_GRAPH=0, which issues the same work directly.
#ifndef PPF_SERVER_GRAPH
#define PPF_SERVER_GRAPH 1
#endif

// Capture the slot's graph for the current class set (scheduler thread, slot idle).
int build_graph(ppf_server_s* s, Slot& sl) {
  if (sl.exec) {
    (void)hipGraphExecDestroy(sl.exec);
    sl.exec = nullptr;
  }
  for (const ClassInfo& ci : s->classes) {
    hipError_t pe = ppf::prepare_desc(ppf_internal_plan_dev(ci.plan), ci.fused);
    if (pe != hipSuccess) return sfail_hip(pe, "descriptor kernel set-up");
  }
  if (!PPF_SERVER_GRAPH) {
    sl.graph_classes = (int)s->classes.size();
    return PPF_OK;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(s->launch, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return sfail_hip(e, "graph capture begin");
  if (e == hipSuccess) e = enqueue_batch(s, sl);
  const int nc = (int)s->classes.size();
  hipError_t e2 = hipStreamEndCapture(s->launch, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return sfail_hip(e != hipSuccess ? e : e2, "graph capture");
  }
  e = hipGraphInstantiate(&sl.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    sl.exec = nullptr;
    return sfail_hip(e, "graph instantiate");
  }
  sl.graph_classes = nc;
  return PPF_OK;
}

// Admit waiting streams in arrival order while the budget allows (caller holds mu).
void admit_waiting(ppf_server_s* s) {
  while (!s->waiting.empty()) {
    auto it = s->streams.find(s->waiting.front());
    if (it == s->streams.end()) {
      s->waiting.pop_front();
      continue;
    }
    SrvStream& st = *it->second;
    if (s->used + st.state_bytes > s->budget) break;
    const size_t hb = (size_t)st.hist_samples * 8;
    bool ok = true;
    for (int i = 0; i < 2 && hb > 0 && ok; ++i) {
      if (hipMalloc(&st.hist[i], hb) != hipSuccess) { st.hist[i] = nullptr; ok = false; }
      else if (hipMemset(st.hist[i], 0, hb) != hipSuccess) ok = false;
    }
    if (!ok) break;   // retried on a later scheduler iteration
    s->used += st.state_bytes;
    st.admitted = true;
    s->stat_admitted++;
    s->order_stale = true;
    s->waiting.pop_front();
  }
}

// Fill slot `sl` from the admitted streams' FIFOs (scheduler thread, mu held).
// Phase 1 picks the chunks: per stream a run of consecutive chunks. The T-1
// blocks before a chunk (its "pre") are kept as at most two memory segments
// (the tail of an older buffer and a short earlier chunk); a run stops where
// the pre of the next chunk would need three. Streams with chunks still in
// flight are skipped when batches run concurrently. The visit starts at a
// rotating stream, so no stream waits behind the others when batches are
// full. Phase 2 cuts the chunks into tiles whose length per plan class
// spreads the class over about kTargetTiles work items. Returns the chunk
// count.
struct Seg {
  const char* p;
  long long n;   // blocks
};
struct Pre {
  Seg s[2];
  int k = 0;     // segments in use
};

// the last `len` blocks of pre (len <= total), as segments
static Pre pre_tail(const Pre& pre, long long len, int N) {
  Pre out;
  long long need = len;
  Seg tmp[2];
  int nt = 0;
  for (int i = pre.k - 1; i >= 0 && need > 0; --i) {
    const long long take = std::min(need, pre.s[i].n);
    tmp[nt++] = Seg{pre.s[i].p + (size_t)(pre.s[i].n - take) * N * 8, take};
    need -= take;
  }
  for (int i = nt - 1; i >= 0; --i) out.s[out.k++] = tmp[i];
  return out;
}

int form_batch(ppf_server_s* s, Slot& sl) {
  DescArea& d = *sl.host;
  const int nc = (int)s->classes.size();
  struct Pick {
    int cls;
    Pre pre;                // the h blocks before the chunk
    ppf_chunk c;
    size_t ws_off;          // two-pass classes: presum offset in the slot workspace
  };
  std::vector<Pick> picks;
  std::vector<long long> cls_spectra(nc, 0);
  int nhist = 0, worst_tiles = 0;
  size_t ws_used = 0;
  sl.chunks.clear();
  if (s->order_stale) {
    s->order.clear();
    for (auto& kv : s->streams)
      if (kv.second->admitted) s->order.push_back(kv.second.get());
    s->order_stale = false;
  }
  const size_t nord = s->order.size();
  const size_t start = nord ? s->rr++ % nord : 0;
  bool full = false;
  for (size_t oi = 0; oi < nord && !full; ++oi) {
    SrvStream& st = *s->order[(start + oi) % nord];
    if (st.queue.empty()) continue;
    if (PPF_SERVER_CONCURRENT_SLOTS && st.inflight > 0) continue;
    const ClassInfo& ci = s->classes[st.cls];
    const int N = ci.N, h = ci.T - 1;
    if (h > 0 && nhist >= kMaxHist) break;
    Pre pre;
    if (h > 0) pre.s[pre.k++] = Seg{(const char*)st.hist[st.cur], h};
    Pre last_pre;
    const void* last_b = nullptr;
    long long last_cs = 0;
    int taken = 0;
    while (!st.queue.empty()) {
      const PendingChunk& pc = st.queue.front();
      const long long S = pc.c.nspectra;
      // tile count at the longest tiles bounds what phase 2 can emit
      const int nt = (int)((S + ci.tile_spectra - 1) / ci.tile_spectra);
      const int ntr = (int)((S + ci.fir_tile_spectra - 1) / ci.fir_tile_spectra);
      const int tiles_needed = ci.fused ? nt : nt + ntr;
      const size_t ws_needed = ci.fused ? 0 : (size_t)S * N * 8;
      if (worst_tiles + tiles_needed > kMaxTiles || ws_used + ws_needed > kSlotWorkspace) {
        full = true;
        break;
      }
      if (pre.k > 2) break;   // this chunk's pre would need three segments
      picks.push_back(Pick{st.cls, pre, pc.c, ws_used});
      cls_spectra[st.cls] += S;
      worst_tiles += tiles_needed;
      ws_used += ws_needed;
      last_pre = pre;
      last_b = pc.c.in;
      last_cs = S * N;
      // the pre of the next chunk: the last h blocks of (pre ++ chunk)
      if (h > 0) {
        if (S >= h) {
          pre = Pre();
          pre.s[pre.k++] = Seg{(const char*)pc.c.in + (size_t)(S - h) * N * 8, h};
        } else {
          Pre next = pre_tail(pre, h - S, N);
          if (next.k < 2) next.s[next.k] = Seg{(const char*)pc.c.in, S};
          next.k++;   // three segments mark a run end (checked before the next chunk)
          pre = next;
        }
      }
      sl.chunks.push_back(DoneChunk{pc.c.tag, pc.arrival_ns, S * N * 8, S, &st, pc.last});
      st.queue.pop_front();
      st.inflight++;
      taken++;
    }
    if (taken == 0) continue;
    if (h > 0) {
      // new history = last h blocks of (last_pre ++ last chunk)
      ppf::HistDesc hd;
      hd.a0 = last_pre.s[0].p;
      hd.n0 = (int)(last_pre.s[0].n * N);
      hd.a1 = last_pre.k > 1 ? (const void*)last_pre.s[1].p : (const void*)last_pre.s[0].p;
      hd.b = last_b;
      hd.dst = st.hist[1 - st.cur];
      hd.hs = (int)(h * N);
      hd.cs = (int)last_cs;
      d.hist[nhist++] = hd;
      st.cur = 1 - st.cur;           // the batch writes the other buffer
    }
  }

  // phase 2: tile lengths per class, then the tiles
  std::vector<int> ts(nc), tsr(nc);
  auto count_tiles = [&]() {
    long long n = 0;
    for (const Pick& pk : picks) {
      const long long S = pk.c.nspectra;
      n += (S + ts[pk.cls] - 1) / ts[pk.cls];
      if (!s->classes[pk.cls].fused) n += (S + tsr[pk.cls] - 1) / tsr[pk.cls];
    }
    return n;
  };
  for (int c = 0; c < nc; ++c) {
    const ClassInfo& ci = s->classes[c];
    const long long want = kTargetTiles > 0 ? (cls_spectra[c] + kTargetTiles - 1) / kTargetTiles : ci.tile_spectra;
    ts[c] = (int)std::max<long long>(1, std::min<long long>(ci.tile_spectra, want));
    tsr[c] = ci.fir_tile_spectra;
  }
  if (count_tiles() > kMaxTiles)
    for (int c = 0; c < nc; ++c) ts[c] = s->classes[c].tile_spectra;   // fits by phase 1
  std::vector<std::vector<ppf::TileDesc>> tf(nc), tr(nc), tt(nc);   // fused, FIR, FFT tiles
  for (const Pick& pk : picks) {
    const ClassInfo& ci = s->classes[pk.cls];
    const int N = ci.N, h = ci.T - 1;
    const long long S = pk.c.nspectra;
    // input tile of spectra m .. m+cnt-1: blocks m .. m+cnt+h-1 of (pre ++ chunk),
    // at most three segments
    auto in_tile = [&](long long m, int cnt) {
      Seg seg[3];
      int k = 0;
      long long skip = m;
      for (int i = 0; i < pk.pre.k; ++i) {
        if (skip >= pk.pre.s[i].n) {
          skip -= pk.pre.s[i].n;
          continue;
        }
        seg[k++] = Seg{pk.pre.s[i].p + (size_t)skip * N * 8, pk.pre.s[i].n - skip};
        skip = 0;
      }
      seg[k++] = Seg{(const char*)pk.c.in + (size_t)skip * N * 8, S + h};   // rest: the chunk
      ppf::TileDesc td;
      td.x0 = seg[0].p;
      td.h0 = k > 1 ? (int)seg[0].n : 0;
      td.x1 = k > 1 ? seg[1].p : seg[0].p;
      td.h1 = k > 2 ? (int)seg[1].n : 0;
      td.x2 = seg[k - 1].p;
      td.count = cnt;
      td.pad_ = 0;
      return td;
    };
    const int t1 = ts[pk.cls];
    if (ci.fused) {
      for (long long m = 0; m < S; m += t1) {
        ppf::TileDesc td = in_tile(m, (int)std::min<long long>(t1, S - m));
        td.out = (char*)pk.c.out + (size_t)m * N * 8;
        tf[pk.cls].push_back(td);
      }
    } else {
      char* u = (char*)sl.ws + pk.ws_off;
      const int t2 = tsr[pk.cls];
      for (long long m = 0; m < S; m += t2) {
        ppf::TileDesc td = in_tile(m, (int)std::min<long long>(t2, S - m));
        td.out = u + (size_t)m * N * 8;
        tr[pk.cls].push_back(td);
      }
      for (long long m = 0; m < S; m += t1) {
        ppf::TileDesc f2;
        f2.x0 = u + (size_t)m * N * 8;
        f2.x1 = f2.x0;
        f2.x2 = f2.x0;
        f2.h0 = 0;
        f2.h1 = 0;
        f2.out = (char*)pk.c.out + (size_t)m * N * 8;
        f2.count = (int)std::min<long long>(t1, S - m);
        f2.pad_ = 0;
        tt[pk.cls].push_back(f2);
      }
    }
  }
  // lay the tiles out class by class
  int at = 0;
  for (int c = 0; c < kMaxClasses; ++c) {
    d.fused[c] = ppf::DescClass{0, 0};
    d.fir[c] = ppf::DescClass{0, 0};
    d.fft[c] = ppf::DescClass{0, 0};
  }
  for (int c = 0; c < nc; ++c) {
    d.fused[c].first = at;
    d.fused[c].ntiles = (int)tf[c].size();
    for (auto& t : tf[c]) d.tiles[at++] = t;
    d.fir[c].first = at;
    d.fir[c].ntiles = (int)tr[c].size();
    for (auto& t : tr[c]) d.tiles[at++] = t;
    d.fft[c].first = at;
    d.fft[c].ntiles = (int)tt[c].size();
    for (auto& t : tt[c]) d.tiles[at++] = t;
  }
  d.nhist = nhist;
  sl.upload_bytes = offsetof(DescArea, tiles) + (size_t)at * sizeof(ppf::TileDesc);
  return (int)sl.chunks.size();
}

// Record the chunks of a finished slot (scheduler thread, mu held).
void complete_slot(ppf_server_s* s, Slot& sl, long long t_done) {
  float ms = 0.f;
  const bool timed = hipEventElapsedTime(&ms, sl.start, sl.done) == hipSuccess;
  long long done = 0;
  {
    std::lock_guard<std::mutex> dl(s->dmu);
    if (timed) {
      s->stat_gpu_us += ms * 1e3;
      s->stat_timed++;
    }
    for (const DoneChunk& dc : sl.chunks) {
      if (dc.last) {
        s->done_tags.push_back(dc.tag);
        if (s->done_tags.size() > kMaxDoneTags) {
          s->done_tags.pop_front();
          s->tags_dropped++;
        }
        s->lat.add((double)(t_done - dc.arrival_ns) * 1e-3);
        s->stat_chunks++;
      }
      s->stat_spectra += dc.spectra;
      s->stat_bytes += dc.bytes;
      if (s->first_arrival < 0 || dc.arrival_ns < s->first_arrival) s->first_arrival = dc.arrival_ns;
    }
    s->last_done = t_done;
  }
  for (const DoneChunk& dc : sl.chunks) {
    dc.stream->outstanding.fetch_sub(1);
    dc.stream->inflight--;
    done++;
  }
  s->outstanding.fetch_sub(done);
  sl.chunks.clear();
  sl.busy = false;
}

// Drop the queued chunks of a stream closed before admission (mu held).
void drop_queue(ppf_server_s* s, SrvStream& st) {
  const long long n = (long long)st.queue.size();
  st.queue.clear();
  st.outstanding.fetch_sub(n);
  s->outstanding.fetch_sub(n);
}

// Slot fields (busy, chunks, exec, host table) belong to the scheduler
// thread; the mutex guards what API threads share with it. HIP calls that
// may take microseconds (graph launch, event query) run unlocked.
void scheduler(ppf_server_s* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    // 1. completions (event queries unlocked)
    int finished[kMaxSlots];
    int nfin = 0;
    bool failed = false;
    lk.unlock();
    for (int k = 0; k < s->nslots; ++k) {
      Slot& sl = s->slots[k];
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipSuccess) finished[nfin++] = k;
      else if (q != hipErrorNotReady) { finished[nfin++] = k; failed = true; }
    }
    const long long t_done = now_ns();
    lk.lock();
    bool progressed = nfin > 0;
    if (failed) s->async_error = PPF_ERR_HIP;
    for (int i = 0; i < nfin; ++i) complete_slot(s, s->slots[finished[i]], t_done);
    // 2. new submissions into the per-stream FIFOs; chunks of streams
    //    closed before admission are dropped
    Submission sub;
    while (s->subq.pop(sub)) {
      SrvStream* st = sub.stream;
      if (st->dropped) {
        st->outstanding.fetch_sub(1);
        s->outstanding.fetch_sub(1);
        progressed = true;
      } else {
        st->queue.push_back(sub.pc);
      }
    }
    bool idle = true;
    for (int k = 0; k < s->nslots; ++k) idle = idle && !s->slots[k].busy;
    // closed streams with nothing left give back their budget now (no
    // batch still refers to them); their buffers are freed when no batch
    // runs, as hipFree may wait for the device
    for (auto it = s->streams.begin(); it != s->streams.end();) {
      SrvStream& st = *it->second;
      if (st.closing && st.outstanding.load() == 0 && st.queue.empty()) {
        if (st.admitted) s->used -= st.state_bytes;
        for (int i = 0; i < 2; ++i)
          if (st.hist[i]) s->deferred_free.push_back(st.hist[i]);
        st.hist[0] = st.hist[1] = nullptr;
        s->waiting.erase(std::remove(s->waiting.begin(), s->waiting.end(), st.id), s->waiting.end());
        it = s->streams.erase(it);
        s->order_stale = true;
        progressed = true;
      } else {
        ++it;
      }
    }
    if (idle && !s->deferred_free.empty()) {
      for (void* p : s->deferred_free) (void)hipFree(p);
      s->deferred_free.clear();
    }
    admit_waiting(s);
    if (s->stop) {
      // shutting down: chunks of streams that were never admitted are dropped
      for (auto& kv : s->streams) {
        SrvStream& st = *kv.second;
        if (!st.admitted && !st.queue.empty()) {
          drop_queue(s, st);
          progressed = true;
        }
      }
    }
    if (progressed) s->cv.notify_all();
    if (s->stop && s->outstanding.load() == 0 && idle && s->subq.empty()) break;
    // 3. launch into a free slot (the next in turn if it is free)
    int free_k = -1;
    for (int i = 0; i < s->nslots && free_k < 0; ++i) {
      const int k = (s->next_slot + i) % s->nslots;
      if (!s->slots[k].busy) free_k = k;
    }
    Slot& sl = s->slots[free_k < 0 ? s->next_slot : free_k];
    bool launched = false;
    if (free_k >= 0 && s->async_error.load() == PPF_OK) {
      bool any_ready = false;
      for (auto& kv : s->streams)
        if (kv.second->admitted && !kv.second->queue.empty()) { any_ready = true; break; }
      if (any_ready && sl.graph_classes != (int)s->classes.size() && idle) {
        for (int k = 0; k < s->nslots; ++k)
          if (build_graph(s, s->slots[k]) != PPF_OK) s->async_error = PPF_ERR_HIP;
      }
      if (any_ready && sl.graph_classes == (int)s->classes.size() && s->async_error.load() == PPF_OK) {
        const long long tf0 = now_ns();
        const int n = form_batch(s, sl);
        if (n > 0) {
          const long long tf1 = now_ns();
          lk.unlock();
          hipStream_t ls = PPF_SERVER_CONCURRENT_SLOTS ? sl.stream : s->launch;
          hipError_t e = hipEventRecord(sl.start, ls);
          if (e == hipSuccess) e = hipMemcpyAsync(sl.dev, sl.host, sl.upload_bytes, hipMemcpyHostToDevice, ls);
          if (e == hipSuccess) e = PPF_SERVER_GRAPH ? hipGraphLaunch(sl.exec, ls) : enqueue_batch(s, sl);
          if (e == hipSuccess) e = hipEventRecord(sl.done, ls);
          const long long tf2 = now_ns();
          lk.lock();
          {
            std::lock_guard<std::mutex> dl(s->dmu);
            s->stat_form_us += (tf1 - tf0) * 1e-3;
            s->stat_launch_us += (tf2 - tf1) * 1e-3;
            s->stat_batches++;
          }
          sl.busy = true;
          s->next_slot = (free_k + 1) % s->nslots;
          if (e != hipSuccess) {
            s->async_error = PPF_ERR_HIP;
            complete_slot(s, sl, now_ns());
          }
          launched = true;
        }
      }
    }
    if (launched) continue;
    // 4. nothing to launch: poll again soon, or sleep until work arrives
    if (!idle) {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else if (!s->stop) {
      // a producer that finds `sleeping` set after its push wakes us; we
      // look at the queue after setting it, so no push is missed
      s->sleeping.store(true);
      if (s->subq.empty()) s->cv.wait_for(lk, std::chrono::microseconds(500));
      s->sleeping.store(false);
    }
  }
}

void destroy_server(ppf_server_s* s) {
  for (int k = 0; k < kMaxSlots; ++k) {
    Slot& sl = s->slots[k];
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    if (sl.stream) {
      (void)hipStreamSynchronize(sl.stream);
      (void)hipStreamDestroy(sl.stream);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.start) (void)hipEventDestroy(sl.start);
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.ws) (void)hipFree(sl.ws);
  }
  for (auto& kv : s->streams) {
    for (int i = 0; i < 2; ++i) {
      if (kv.second->hist[i]) (void)hipFree(kv.second->hist[i]);
      kv.second->hist[i] = nullptr;
    }
  }
  for (void* p : s->deferred_free) (void)hipFree(p);
  for (ppf_stream_s* h : s->handles) h->server = nullptr;   // orphaned: only ppf_stream_destroy remains
  for (int c = 0; c < kMaxClasses; ++c) {
    if (s->branch[c]) (void)hipStreamDestroy(s->branch[c]);
    if (s->join[c]) (void)hipEventDestroy(s->join[c]);
  }
  if (s->hist_branch) (void)hipStreamDestroy(s->hist_branch);
  if (s->hist_join) (void)hipEventDestroy(s->hist_join);
  if (s->fork) (void)hipEventDestroy(s->fork);
  if (s->launch) (void)hipStreamDestroy(s->launch);
  delete s;
}

// Wake the scheduler if it sleeps (after a push).
void wake(ppf_server_s* s) {
  if (s->sleeping.load()) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv.notify_all();
  }
}

int open_stream(ppf_server_s* s, ppf_plan_t plan, int flags, ppf_stream_t* out) {
  if (!s || !plan || !out) return sfail(PPF_ERR_INVALID, "server, plan or out is NULL");
  if (flags & ~PPF_OPEN_NOWAIT) return sfail(PPF_ERR_INVALID, "unknown flags %d", flags);
  long long in_type = -1, N = 0, T = 0, fft = 0;
  ppf_plan_query(plan, PPF_Q_IN_TYPE, &in_type);
  ppf_plan_query(plan, PPF_Q_N, &N);
  ppf_plan_query(plan, PPF_Q_TAPS, &T);
  ppf_plan_query(plan, PPF_Q_FFT_MODE, &fft);
  if (in_type != PPF_C32 || fft != PPF_FFT_F32)
    return sfail(PPF_ERR_UNSUPPORTED, "the server takes complex FP32 plans with FP32 DFT stages");
  std::unique_ptr<ppf_stream_s> h(new (std::nothrow) ppf_stream_s);
  if (!h) return sfail(PPF_ERR_NOMEM, "host allocation");
  const size_t state = stream_state_bytes((int)N, (int)T);
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stop) return sfail(PPF_ERR_INVALID, "server is shutting down");
  const size_t fixed = (size_t)s->nslots * (sizeof(DescArea) + kSlotWorkspace);
  if (fixed + state > s->budget) {
    s->stat_rejected++;
    return sfail(PPF_ERR_BUDGET, "stream state of %zu bytes can never fit the budget", state);
  }
  const bool fits = s->waiting.empty() && s->used + state <= s->budget;
  if (!fits && (flags & PPF_OPEN_NOWAIT)) {
    s->stat_rejected++;
    return sfail(PPF_ERR_BUDGET, "stream state of %zu bytes exceeds the remaining budget", state);
  }
  const int cls = class_of(s, plan);
  if (cls < 0) return sfail(PPF_ERR_UNSUPPORTED, "more than %d plans in one server", kMaxClasses);
  auto st = std::make_shared<SrvStream>();
  st->id = s->next_id++;
  st->plan = plan;
  st->cls = cls;
  st->N = (int)N;
  st->max_piece = s->classes[cls].max_piece;
  st->hist_samples = (T - 1) * N;
  st->state_bytes = state;
  s->streams[st->id] = st;
  s->waiting.push_back(st->id);
  if (!fits) s->stat_queued++;
  admit_waiting(s);
  h->plan = plan;
  h->server_stream = true;
  h->server = s;
  h->srv = st;
  h->hist_samples = st->hist_samples;
  s->handles.insert(h.get());
  *out = h.release();
  s->cv.notify_all();
  return PPF_OK;
}

}  // namespace

// A push to a server stream: the chunk goes to the submission queue, in
// pieces an empty batch can hold (only the last piece reports the tag).
int ppf_internal_server_push(ppf_stream_s* h, const ppf_chunk* chunk, long long arrival_ns) {
  if (!h || !chunk) return sfail(PPF_ERR_INVALID, "stream or chunk is NULL");
  ppf_server_s* s = h->server;
  if (!s) return sfail(PPF_ERR_INVALID, "the stream's server was destroyed");
  SrvStream* st = h->srv.get();
  const long long S = chunk->nspectra;
  if (S < 0) return sfail(PPF_ERR_INVALID, "nspectra=%lld is negative", S);
  if (S == 0) return PPF_OK;
  if (S > kMaxChunkSpectra) return sfail(PPF_ERR_INVALID, "nspectra=%lld exceeds 2^31", S);
  if (!chunk->in || !chunk->out) return sfail(PPF_ERR_INVALID, "chunk in or out is NULL");
  if (((uintptr_t)chunk->in & 15) || ((uintptr_t)chunk->out & 15))
    return sfail(PPF_ERR_ALIGN, "chunk in and out must be 16-byte aligned");
  if (st->closing.load()) return sfail(PPF_ERR_INVALID, "stream %d is closed", st->id);
  if (s->async_error.load() != PPF_OK) return sfail(s->async_error.load(), "server failed earlier");
  const long long N = st->N;
  const size_t in_b = (size_t)S * N * 8;
  if ((uintptr_t)chunk->in < (uintptr_t)chunk->out + in_b && (uintptr_t)chunk->out < (uintptr_t)chunk->in + in_b)
    return sfail(PPF_ERR_INVALID, "chunk in and out overlap");
  const long long piece = st->max_piece;
  const long long t = arrival_ns >= 0 ? arrival_ns : now_ns();
  for (long long m0 = 0; m0 < S; m0 += piece) {
    const long long k = std::min(piece, S - m0);
    Submission sub;
    sub.stream = st;
    sub.pc.c.in = (const char*)chunk->in + (size_t)m0 * N * 8;
    sub.pc.c.out = (char*)chunk->out + (size_t)m0 * N * 8;
    sub.pc.c.nspectra = k;
    sub.pc.c.tag = chunk->tag;
    sub.pc.arrival_ns = t;
    sub.pc.last = m0 + k == S;
    st->outstanding.fetch_add(1);
    s->outstanding.fetch_add(1);
    while (!s->subq.push(sub)) {   // full: the scheduler is behind
      wake(s);
      std::this_thread::yield();
    }
  }
  h->pushed_spectra += S;
  wake(s);
  return PPF_OK;
}

// Destroying a server stream closes it, waits until its chunks are done
// (or the server failed) and frees the handle.
int ppf_internal_server_stream_destroy(ppf_stream_s* h) {
  ppf_server_s* s = h->server;
  int rc = PPF_OK;
  if (s) {
    SrvStream* st = h->srv.get();
    std::unique_lock<std::mutex> lk(s->mu);
    st->closing = true;
    if (!st->admitted) {
      st->dropped = true;
      s->waiting.erase(std::remove(s->waiting.begin(), s->waiting.end(), st->id), s->waiting.end());
      drop_queue(s, *st);
    }
    s->cv.notify_all();
    while (st->outstanding.load() > 0 && s->async_error.load() == PPF_OK && !s->stop.load())
      s->cv.wait_for(lk, std::chrono::milliseconds(50));
    if (st->outstanding.load() > 0) rc = sfail(s->async_error.load() != PPF_OK ? s->async_error.load() : PPF_ERR_BUSY,
                                               "stream %d still had chunks when it was destroyed", st->id);
    s->handles.erase(h);
  }
  delete h;
  return rc;
}

extern "C" {

long long ppf_clock_ns(void) { return now_ns(); }

ppf_server_t ppf_server_create(size_t hbm_budget_bytes, int max_inflight) {
  if (max_inflight < 1 || max_inflight > kMaxSlots) {
    sfail(PPF_ERR_INVALID, "max_inflight=%d outside 1..%d", max_inflight, kMaxSlots);
    return nullptr;
  }
  const size_t fixed = (size_t)max_inflight * (sizeof(DescArea) + kSlotWorkspace);
  if (hbm_budget_bytes < fixed) {
    sfail(PPF_ERR_BUDGET, "budget %zu below the server's own %zu bytes", hbm_budget_bytes, fixed);
    return nullptr;
  }
  ppf_server_s* s = new (std::nothrow) ppf_server_s;
  if (!s) { sfail(PPF_ERR_NOMEM, "host allocation"); return nullptr; }
  s->budget = hbm_budget_bytes;
  s->used = fixed;
  s->nslots = max_inflight;
  hipError_t e = hipStreamCreateWithFlags(&s->launch, hipStreamNonBlocking);
  for (int c = 0; c < kMaxClasses && e == hipSuccess; ++c) {
    e = hipStreamCreateWithFlags(&s->branch[c], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->join[c], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->hist_branch, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->hist_join, hipEventDisableTiming);
  for (int k = 0; k < s->nslots && e == hipSuccess; ++k) {
    Slot& sl = s->slots[k];
    e = hipHostMalloc((void**)&sl.host, sizeof(DescArea), hipHostMallocDefault);
    if (e == hipSuccess) std::memset(sl.host, 0, sizeof(DescArea));
    if (e == hipSuccess) e = hipMalloc((void**)&sl.dev, sizeof(DescArea));
    if (e == hipSuccess) e = hipMalloc(&sl.ws, kSlotWorkspace);
    if (e == hipSuccess) e = hipEventCreate(&sl.done);
    if (e == hipSuccess) e = hipEventCreate(&sl.start);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
  }
  if (e != hipSuccess) {
    sfail_hip(e, "server creation");
    destroy_server(s);
    return nullptr;
  }
  try {
    s->worker = std::thread(scheduler, s);
  } catch (...) {
    sfail(PPF_ERR_NOMEM, "scheduler thread");
    destroy_server(s);
    return nullptr;
  }
  return s;
}

int ppf_server_open_stream(ppf_server_t s, ppf_plan_t plan, ppf_stream_t* out) {
  try {
    return open_stream(s, plan, 0, out);
  } catch (...) {
    return sfail(PPF_ERR_NOMEM, "unexpected exception in ppf_server_open_stream");
  }
}

int ppf_server_open_stream_ex(ppf_server_t s, ppf_plan_t plan, int flags, ppf_stream_t* out) {
  try {
    return open_stream(s, plan, flags, out);
  } catch (...) {
    return sfail(PPF_ERR_NOMEM, "unexpected exception in ppf_server_open_stream_ex");
  }
}

int ppf_server_stream_admitted(ppf_stream_t stream) {
  if (!stream || !stream->server_stream) return sfail(PPF_ERR_INVALID, "not a server stream");
  if (!stream->server) return sfail(PPF_ERR_INVALID, "the stream's server was destroyed");
  return stream->srv->admitted.load() ? 1 : 0;
}

int ppf_server_submit(ppf_stream_t stream, const ppf_chunk* chunk, long long arrival_ns) {
  if (!stream || !stream->server_stream) return sfail(PPF_ERR_INVALID, "not a server stream");
  try {
    return ppf_internal_server_push(stream, chunk, arrival_ns);
  } catch (...) {
    return sfail(PPF_ERR_NOMEM, "unexpected exception in ppf_server_submit");
  }
}

int ppf_server_poll(ppf_server_t s, unsigned long long* tags, int max) {
  if (!s || (!tags && max > 0) || max < 0) return sfail(PPF_ERR_INVALID, "bad arguments");
  std::lock_guard<std::mutex> lk(s->dmu);
  int n = 0;
  while (n < max && !s->done_tags.empty()) {
    tags[n++] = s->done_tags.front();
    s->done_tags.pop_front();
  }
  return n;
}

int ppf_server_drain(ppf_server_t s, double timeout_s) {
  if (!s) return sfail(PPF_ERR_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                            std::chrono::duration<double>(timeout_s));
  while (s->outstanding.load() > 0) {
    if (s->async_error.load() != PPF_OK) return sfail(s->async_error.load(), "server failed");
    s->cv.wait_until(lk, std::min(deadline, std::chrono::steady_clock::now() + std::chrono::milliseconds(20)));
    if (std::chrono::steady_clock::now() >= deadline && s->outstanding.load() > 0)
      return sfail(PPF_ERR_BUSY, "%lld chunks still outstanding", s->outstanding.load());
  }
  return s->async_error.load() == PPF_OK ? PPF_OK : sfail(s->async_error.load(), "server failed");
}

int ppf_server_close_stream(ppf_stream_t stream) {
  if (!stream || !stream->server_stream) return sfail(PPF_ERR_INVALID, "not a server stream");
  ppf_server_s* s = stream->server;
  if (!s) return sfail(PPF_ERR_INVALID, "the stream's server was destroyed");
  SrvStream* st = stream->srv.get();
  std::lock_guard<std::mutex> lk(s->mu);
  st->closing = true;
  if (!st->admitted) {
    // never admitted: leave the waiting line now; its queued chunks, and
    // any still on their way to the scheduler, are dropped
    st->dropped = true;
    s->waiting.erase(std::remove(s->waiting.begin(), s->waiting.end(), st->id), s->waiting.end());
    drop_queue(s, *st);
  }
  s->cv.notify_all();
  return PPF_OK;
}

int ppf_server_get_stats(ppf_server_t s, ppf_server_stats_t* out) {
  if (!s || !out) return sfail(PPF_ERR_INVALID, "server or out is NULL");
  std::memset(out, 0, sizeof *out);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    out->admitted = s->stat_admitted;
    out->rejected = s->stat_rejected;
    out->queued_admissions = s->stat_queued;
    out->state_bytes_used = (long long)s->used;
  }
  std::lock_guard<std::mutex> dl(s->dmu);
  out->chunks_done = s->stat_chunks;
  out->spectra_done = s->stat_spectra;
  out->bytes_in_done = s->stat_bytes;
  out->batches = s->stat_batches;
  out->tags_dropped = s->tags_dropped;
  if (s->lat.count() > 0) {
    out->p50_us = s->lat.pct(0.50);
    out->p99_us = s->lat.pct(0.99);
    out->max_us = s->lat.max();
    out->mean_us = s->lat.mean();
  }
  if (s->first_arrival >= 0 && s->last_done > s->first_arrival) {
    out->elapsed_s = (s->last_done - s->first_arrival) * 1e-9;
    out->input_gbps = s->stat_bytes / out->elapsed_s / 1e9;
  }
  out->mean_batch_chunks = s->stat_batches ? (double)s->stat_chunks / s->stat_batches : 0.0;
  out->mean_batch_gpu_us = s->stat_timed ? s->stat_gpu_us / s->stat_timed : 0.0;
  out->mean_form_us = s->stat_batches ? s->stat_form_us / s->stat_batches : 0.0;
  out->mean_launch_us = s->stat_batches ? s->stat_launch_us / s->stat_batches : 0.0;
  return PPF_OK;
}

int ppf_server_stats(ppf_server_t s, double* p50_us, double* p99_us, double* gbps) {
  ppf_server_stats_t st;
  const int rc = ppf_server_get_stats(s, &st);
  if (rc != PPF_OK) return rc;
  if (p50_us) *p50_us = st.p50_us;
  if (p99_us) *p99_us = st.p99_us;
  if (gbps) *gbps = st.input_gbps;
  return PPF_OK;
}

int ppf_server_reset_stats(ppf_server_t s) {
  if (!s) return sfail(PPF_ERR_INVALID, "server is NULL");
  std::lock_guard<std::mutex> dl(s->dmu);
  s->lat.clear();
  s->stat_gpu_us = s->stat_form_us = s->stat_launch_us = 0;
  s->stat_timed = 0;
  s->stat_chunks = s->stat_spectra = s->stat_bytes = s->stat_batches = 0;
  s->first_arrival = s->last_done = -1;
  return PPF_OK;
}

int ppf_server_destroy(ppf_server_t s) {
  if (!s) return PPF_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  const int err = s->async_error.load();
  for (int k = 0; k < s->nslots; ++k)
    if (s->slots[k].stream) (void)hipStreamSynchronize(s->slots[k].stream);
  (void)hipStreamSynchronize(s->launch);
  destroy_server(s);
  return err == PPF_OK ? PPF_OK : sfail(err, "server had failed");
}

}  // extern "C"

// Serving form of libppf.so: continuous batching of chunks from many
// streams of different N and T onto the GPU.
//
// Producers submit chunks from any thread. One scheduler thread per server
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
#include <cstddef>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
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
};

struct SrvStream {
  int id = -1;
  ppf_plan_t plan = nullptr;
  int cls = -1;
  void* hist[2] = {nullptr, nullptr};
  int cur = 0;
  long long hist_samples = 0;
  size_t state_bytes = 0;
  bool admitted = false;
  bool closing = false;
  std::deque<PendingChunk> queue;   // scheduler-owned
  long long outstanding = 0;        // submitted, not completed
  long long inflight = 0;           // in a launched batch, not completed (scheduler-owned)
};

struct DoneChunk {
  unsigned long long tag;
  long long arrival_ns;
  long long bytes;
  long long spectra;
  int stream;
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
};

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
  size_t used = 0;                 // state bytes of admitted streams + fixed buffers
  int nslots = 2;
  Slot slots[kMaxSlots];
  int next_slot = 0;               // the slot launched next (launch order = completion order)
  hipStream_t launch = nullptr;
  hipStream_t branch[kMaxClasses] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxClasses] = {};
  hipStream_t hist_branch = nullptr;   // history updates of a batch
  hipEvent_t hist_join = nullptr;

  std::mutex mu;                   // guards everything below
  std::condition_variable cv;      // wakes the scheduler, signals drains
  std::vector<ClassInfo> classes;
  std::map<int, std::unique_ptr<SrvStream>> streams;
  std::deque<int> waiting;         // streams waiting for admission, in order
  std::vector<std::pair<int, PendingChunk>> pending;
  std::deque<unsigned long long> done_tags;
  std::vector<double> lat_us;
  long long stat_chunks = 0, stat_spectra = 0, stat_bytes = 0, stat_batches = 0;
  long long stat_admitted = 0, stat_rejected = 0, stat_queued = 0;
  double stat_gpu_us = 0, stat_form_us = 0, stat_launch_us = 0;
  long long stat_timed = 0;
  long long first_arrival = -1, last_done = -1;
  long long outstanding = 0;       // submitted, not completed, all streams
  int next_id = 0;
  int async_error = PPF_OK;
  bool stop = false;
  std::thread worker;
};

namespace {

size_t stream_state_bytes(int N, int T) { return 2ull * (size_t)(T - 1) * N * 8 + 4096; }

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
  // tiles of about 32K samples, 4..64 spectra
  int ts = 32768 / ci.N;
  ci.tile_spectra = ts < 4 ? 4 : (ts > 64 ? 64 : ts);
  s->classes.push_back(ci);
  return (int)s->classes.size() - 1;
}

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
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(s->launch, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return sfail_hip(e, "graph capture begin");
  // the descriptor upload precedes each launch (only the used bytes)
  e = hipEventRecord(s->fork, s->launch);
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
    s->waiting.pop_front();
  }
}

// Fill slot `sl` from the admitted streams' FIFOs (scheduler thread, mu held).
// Phase 1 picks the chunks: per stream a run of consecutive chunks. The T-1
// blocks before a chunk (its "pre") are kept as at most two memory segments
// (the tail of an older buffer and a short earlier chunk); a run stops where
// the pre of the next chunk would need three. Streams with chunks still in
// flight are skipped when batches run concurrently. Phase 2 cuts the chunks
// into tiles whose length per plan class spreads the class over about
// kTargetTiles work items. Returns the chunk count.
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
  for (auto& kv : s->streams) {
    SrvStream& st = *kv.second;
    if (!st.admitted || st.queue.empty()) continue;
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
      if (worst_tiles + tiles_needed > kMaxTiles || ws_used + ws_needed > kSlotWorkspace) break;
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
      sl.chunks.push_back(DoneChunk{pc.c.tag, pc.arrival_ns, S * N * 8, S, st.id});
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

// Record the chunks of a finished slot (mu held).
void complete_slot(ppf_server_s* s, Slot& sl, long long t_done) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, sl.start, sl.done) == hipSuccess) {
    s->stat_gpu_us += ms * 1e3;
    s->stat_timed++;
  }
  for (const DoneChunk& dc : sl.chunks) {
    s->done_tags.push_back(dc.tag);
    s->lat_us.push_back((double)(t_done - dc.arrival_ns) * 1e-3);
    s->stat_chunks++;
    s->stat_spectra += dc.spectra;
    s->stat_bytes += dc.bytes;
    if (s->first_arrival < 0 || dc.arrival_ns < s->first_arrival) s->first_arrival = dc.arrival_ns;
    auto it = s->streams.find(dc.stream);
    if (it != s->streams.end()) {
      it->second->outstanding--;
      it->second->inflight--;
    }
    s->outstanding--;
  }
  s->last_done = t_done;
  sl.chunks.clear();
  sl.busy = false;
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
    // 2. new submissions into the per-stream FIFOs
    if (!s->pending.empty()) {
      for (auto& pr : s->pending) {
        auto it = s->streams.find(pr.first);
        if (it != s->streams.end()) it->second->queue.push_back(pr.second);
      }
      s->pending.clear();
    }
    bool idle = true;
    for (int k = 0; k < s->nslots; ++k) idle = idle && !s->slots[k].busy;
    // closed streams with nothing left release their state once no batch runs
    if (idle) {
      for (auto it = s->streams.begin(); it != s->streams.end();) {
        SrvStream& st = *it->second;
        if (st.closing && st.outstanding == 0 && st.queue.empty()) {
          if (st.admitted) s->used -= st.state_bytes;
          if (st.hist[0]) (void)hipFree(st.hist[0]);
          if (st.hist[1]) (void)hipFree(st.hist[1]);
          it = s->streams.erase(it);
          progressed = true;
        } else {
          ++it;
        }
      }
    }
    admit_waiting(s);
    if (s->stop) {
      // shutting down: chunks of streams that were never admitted are dropped
      for (auto& kv : s->streams) {
        SrvStream& st = *kv.second;
        if (!st.admitted && !st.queue.empty()) {
          s->outstanding -= (long long)st.queue.size();
          st.outstanding -= (long long)st.queue.size();
          st.queue.clear();
          progressed = true;
        }
      }
    }
    if (progressed) s->cv.notify_all();
    if (s->stop && s->outstanding == 0 && idle) break;
    // 3. launch into a free slot (the next in turn if it is free)
    int free_k = -1;
    for (int i = 0; i < s->nslots && free_k < 0; ++i) {
      const int k = (s->next_slot + i) % s->nslots;
      if (!s->slots[k].busy) free_k = k;
    }
    Slot& sl = s->slots[free_k < 0 ? s->next_slot : free_k];
    bool launched = false;
    if (free_k >= 0 && s->async_error == PPF_OK) {
      bool any_ready = false;
      for (auto& kv : s->streams)
        if (kv.second->admitted && !kv.second->queue.empty()) { any_ready = true; break; }
      if (any_ready && sl.graph_classes != (int)s->classes.size() && idle) {
        for (int k = 0; k < s->nslots; ++k)
          if (build_graph(s, s->slots[k]) != PPF_OK) s->async_error = PPF_ERR_HIP;
      }
      if (any_ready && sl.graph_classes == (int)s->classes.size() && s->async_error == PPF_OK) {
        const long long tf0 = now_ns();
        const int n = form_batch(s, sl);
        if (n > 0) {
          const long long tf1 = now_ns();
          lk.unlock();
          hipStream_t ls = PPF_SERVER_CONCURRENT_SLOTS ? sl.stream : s->launch;
          hipError_t e = hipEventRecord(sl.start, ls);
          if (e == hipSuccess) e = hipMemcpyAsync(sl.dev, sl.host, sl.upload_bytes, hipMemcpyHostToDevice, ls);
          if (e == hipSuccess) e = hipGraphLaunch(sl.exec, ls);
          if (e == hipSuccess) e = hipEventRecord(sl.done, ls);
          const long long tf2 = now_ns();
          lk.lock();
          s->stat_form_us += (tf1 - tf0) * 1e-3;
          s->stat_launch_us += (tf2 - tf1) * 1e-3;
          sl.busy = true;
          s->stat_batches++;
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
    } else if (s->pending.empty() && !s->stop) {
      s->cv.wait_for(lk, std::chrono::microseconds(500));
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
    if (kv.second->hist[0]) (void)hipFree(kv.second->hist[0]);
    if (kv.second->hist[1]) (void)hipFree(kv.second->hist[1]);
  }
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

}  // namespace

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

int ppf_server_open_stream(ppf_server_t s, ppf_plan_t plan, int wait_for_budget, int* stream_id) {
  if (!s || !plan || !stream_id) return sfail(PPF_ERR_INVALID, "server, plan or stream_id is NULL");
  long long in_type = -1, N = 0, T = 0;
  ppf_plan_query(plan, PPF_Q_IN_TYPE, &in_type);
  ppf_plan_query(plan, PPF_Q_N, &N);
  ppf_plan_query(plan, PPF_Q_TAPS, &T);
  if (in_type != PPF_C32) return sfail(PPF_ERR_UNSUPPORTED, "the server takes complex FP32 plans");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stop) return sfail(PPF_ERR_INVALID, "server is shutting down");
  const int cls = class_of(s, plan);
  if (cls < 0) return sfail(PPF_ERR_UNSUPPORTED, "more than %d plans in one server", kMaxClasses);
  auto st = std::make_unique<SrvStream>();
  st->id = s->next_id++;
  st->plan = plan;
  st->cls = cls;
  st->hist_samples = (T - 1) * N;
  st->state_bytes = stream_state_bytes((int)N, (int)T);
  const bool fits = s->waiting.empty() && s->used + st->state_bytes <= s->budget;
  if (!fits && !wait_for_budget) {
    s->stat_rejected++;
    return sfail(PPF_ERR_BUDGET, "stream state of %zu bytes exceeds the remaining budget", st->state_bytes);
  }
  const int id = st->id;
  s->streams[id] = std::move(st);
  s->waiting.push_back(id);
  if (!fits) s->stat_queued++;
  admit_waiting(s);
  *stream_id = id;
  s->cv.notify_all();
  return PPF_OK;
}

int ppf_server_stream_admitted(ppf_server_t s, int stream_id) {
  if (!s) return sfail(PPF_ERR_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->streams.find(stream_id);
  if (it == s->streams.end()) return sfail(PPF_ERR_INVALID, "unknown stream %d", stream_id);
  return it->second->admitted ? 1 : 0;
}

int ppf_server_submit(ppf_server_t s, int stream_id, const ppf_chunk* chunk, long long arrival_ns) {
  if (!s || !chunk) return sfail(PPF_ERR_INVALID, "server or chunk is NULL");
  if (chunk->nspectra <= 0) return sfail(PPF_ERR_INVALID, "nspectra=%lld must be positive", chunk->nspectra);
  if (!chunk->in || !chunk->out) return sfail(PPF_ERR_INVALID, "chunk in or out is NULL");
  if (((uintptr_t)chunk->in & 15) || ((uintptr_t)chunk->out & 15))
    return sfail(PPF_ERR_ALIGN, "chunk in and out must be 16-byte aligned");
  const long long t = arrival_ns >= 0 ? arrival_ns : now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->streams.find(stream_id);
  if (it == s->streams.end() || it->second->closing) return sfail(PPF_ERR_INVALID, "stream %d is not open", stream_id);
  if (s->async_error != PPF_OK) return sfail(s->async_error, "server failed earlier");
  const ClassInfo& ci = s->classes[it->second->cls];
  if (chunk->nspectra > (1ll << 24)) return sfail(PPF_ERR_INVALID, "chunk too large");
  const size_t in_b = (size_t)chunk->nspectra * ci.N * 8;
  if ((uintptr_t)chunk->in < (uintptr_t)chunk->out + in_b && (uintptr_t)chunk->out < (uintptr_t)chunk->in + in_b)
    return sfail(PPF_ERR_INVALID, "chunk in and out overlap");
  s->pending.emplace_back(stream_id, PendingChunk{*chunk, t});
  it->second->outstanding++;
  s->outstanding++;
  s->cv.notify_all();
  return PPF_OK;
}

int ppf_server_poll(ppf_server_t s, unsigned long long* tags, int max) {
  if (!s || (!tags && max > 0) || max < 0) return sfail(PPF_ERR_INVALID, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
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
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  while (s->outstanding > 0) {
    if (s->async_error != PPF_OK) return sfail(s->async_error, "server failed");
    if (s->cv.wait_until(lk, deadline) == std::cv_status::timeout && s->outstanding > 0)
      return sfail(PPF_ERR_BUSY, "%lld chunks still outstanding", s->outstanding);
  }
  return s->async_error == PPF_OK ? PPF_OK : sfail(s->async_error, "server failed");
}

int ppf_server_close_stream(ppf_server_t s, int stream_id) {
  if (!s) return sfail(PPF_ERR_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->streams.find(stream_id);
  if (it == s->streams.end()) return sfail(PPF_ERR_INVALID, "unknown stream %d", stream_id);
  it->second->closing = true;
  if (!it->second->admitted) {
    // never admitted: drop it from the waiting line now
    s->waiting.erase(std::remove(s->waiting.begin(), s->waiting.end(), stream_id), s->waiting.end());
    it->second->queue.clear();
  }
  s->cv.notify_all();
  return PPF_OK;
}

int ppf_server_get_stats(ppf_server_t s, ppf_server_stats* out) {
  if (!s || !out) return sfail(PPF_ERR_INVALID, "server or out is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof *out);
  out->chunks_done = s->stat_chunks;
  out->spectra_done = s->stat_spectra;
  out->bytes_in_done = s->stat_bytes;
  out->batches = s->stat_batches;
  out->admitted = s->stat_admitted;
  out->rejected = s->stat_rejected;
  out->queued_admissions = s->stat_queued;
  out->state_bytes_used = (long long)s->used;
  if (!s->lat_us.empty()) {
    std::vector<double> v = s->lat_us;
    auto pct = [&](double p) {
      size_t k = (size_t)(p * (v.size() - 1) + 0.5);
      std::nth_element(v.begin(), v.begin() + k, v.end());
      return v[k];
    };
    out->p50_us = pct(0.50);
    out->p99_us = pct(0.99);
    out->max_us = *std::max_element(v.begin(), v.end());
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_us = sum / v.size();
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

int ppf_server_reset_stats(ppf_server_t s) {
  if (!s) return sfail(PPF_ERR_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat_us.clear();
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
  const int err = s->async_error;
  for (int k = 0; k < s->nslots; ++k)
    if (s->slots[k].stream) (void)hipStreamSynchronize(s->slots[k].stream);
  (void)hipStreamSynchronize(s->launch);
  destroy_server(s);
  return err == PPF_OK ? PPF_OK : sfail(err, "server had failed");
}

}  // extern "C"

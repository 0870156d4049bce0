// C ABI of the IDBF library (include/idbf.h): argument checks, the level
// schedule of the construction, factor memory, the apply stage sequence,
// inspection and the stand-alone sampler / ID entry points.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace idbf {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
  int l = 0;
  while ((1ll << l) < v) ++l;
  return l;
}

// Device memory of released handles, kept for later ones on the same device.
// A construction makes several large hipMalloc calls and its handle as many
// hipFree calls, and on this platform each can take from milliseconds to
// seconds.  Chunks enter only when the device is idle (release synchronizes
// it), so a reused chunk has no work in flight.  Bounded by IDBF_CACHE_BYTES
// (default 32 GiB, 0 disables; the oldest chunks are freed first);
// idbf_release_cached_memory frees everything held.
struct ChunkCache {
  struct Entry {
    int dev;
    void* p;
    size_t size;
  };
  std::mutex mu;
  std::vector<Entry> list;  // oldest first
  size_t held = 0, cap = 0;
  std::vector<void*> pinned;  // HostStage-sized pinned blocks
  size_t pinned_size = 0;

  ChunkCache() {
    cap = size_t(32) << 30;
    if (const char* e = std::getenv("IDBF_CACHE_BYTES")) cap = (size_t)std::strtoull(e, nullptr, 10);
  }
  // the smallest held chunk of [want, min(4 want, most)] bytes on device dev, or null
  void* take(int dev, size_t want, size_t most, size_t* got) {
    std::lock_guard<std::mutex> g(mu);
    int best = -1;
    for (size_t i = 0; i < list.size(); ++i) {
      const Entry& e = list[i];
      if (e.dev == dev && e.size >= want && e.size <= most && e.size / 4 <= want &&
          (best < 0 || e.size < list[best].size))
        best = (int)i;
    }
    if (best < 0) return nullptr;
    const Entry e = list[best];
    list.erase(list.begin() + best);
    held -= e.size;
    *got = e.size;
    return e.p;
  }
  // an idle chunk back; chunks past the bound are freed
  void put(int dev, void* p, size_t size) {
    std::vector<Entry> drop;
    {
      std::lock_guard<std::mutex> g(mu);
      if (size > cap) {
        drop.push_back({dev, p, size});
      } else {
        list.push_back({dev, p, size});
        held += size;
        while (held > cap) {
          drop.push_back(list.front());
          held -= list.front().size;
          list.erase(list.begin());
        }
      }
    }
    for (const Entry& e : drop) (void)hipFree(e.p);
  }
  void* take_pinned(size_t size) {
    std::lock_guard<std::mutex> g(mu);
    if (pinned.empty() || pinned_size != size) return nullptr;
    void* p = pinned.back();
    pinned.pop_back();
    return p;
  }
  void put_pinned(void* p, size_t size) {
    {
      std::lock_guard<std::mutex> g(mu);
      if (cap > 0 && pinned.size() < 256 && (pinned.empty() || pinned_size == size)) {
        pinned_size = size;
        pinned.push_back(p);
        return;
      }
    }
    (void)hipHostFree(p);
  }
  void clear() {
    std::vector<Entry> drop;
    std::vector<void*> pins;
    {
      std::lock_guard<std::mutex> g(mu);
      drop.swap(list);
      pins.swap(pinned);
      held = 0;
    }
    for (const Entry& e : drop) (void)hipFree(e.p);
    for (void* p : pins) (void)hipHostFree(p);
  }
};

// never destroyed: freeing device memory while the process exits is not safe
ChunkCache& chunk_cache() {
  static ChunkCache* c = new ChunkCache;
  return *c;
}

int current_device() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) {
    (void)hipGetLastError();
    d = 0;
  }
  return d;
}

// Device memory of at least `bytes` and at most `most` (a held chunk when one
// fits), its size in *got.
hipError_t device_alloc(size_t bytes, size_t most, void** p, size_t* got) {
  if (void* q = chunk_cache().take(current_device(), bytes, most, got)) {
    *p = q;
    return hipSuccess;
  }
  *got = bytes;
  return hipMalloc(p, bytes);
}

// A handle's device memory: the caller's allocator (opts.dev_alloc /
// dev_free) when it gave one, else hipMalloc behind the chunk cache.
struct Allocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, size_t, void*) = nullptr;
  void* user = nullptr;

  hipError_t get(size_t bytes, size_t most, void** p, size_t* got) const {
    if (!alloc) return device_alloc(bytes, most, p, got);
    void* q = alloc(bytes, user);
    if (!q) return hipErrorOutOfMemory;
    *p = q;
    *got = bytes;
    return hipSuccess;
  }
  // back to the caller, or to the cache; the device must be done with it
  void put(int dev, void* p, size_t bytes) const {
    if (free) free(p, bytes, user);
    else chunk_cache().put(dev, p, bytes);
  }
};

// Bump allocator over large device chunks: the construction's many per-level
// arrays cost a handful of allocations.
struct Arena {
  struct Chunk {
    void* base;
    size_t size;
    int dev;
  };
  std::vector<Chunk> chunks;
  char* cur = nullptr;
  size_t used = 0, cap = 0, total = 0, limit = 0, chunk_min = size_t(64) << 20;
  Allocator al;

  idbf_status alloc(size_t bytes, void** out) {
    bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
    if (cur && used + bytes <= cap) {
      *out = cur + used;
      used += bytes;
      return IDBF_OK;
    }
    size_t sz = std::max(bytes, chunk_min);
    if (limit && total + sz > limit) sz = bytes;
    if (limit && total + sz > limit) {
      set_error("device memory cap of %zu bytes exceeded (%zu held, %zu requested)", limit, total, bytes);
      return IDBF_ENOMEM;
    }
    void* p = nullptr;
    size_t got = sz;
    hipError_t e = al.get(sz, limit ? limit - total : SIZE_MAX, &p, &got);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("device allocation of %zu bytes failed: %s", sz, hipGetErrorString(e));
      return IDBF_ENOMEM;
    }
    chunks.push_back({p, got, current_device()});
    total += got;
    cur = static_cast<char*>(p);
    used = bytes;
    cap = got;
    *out = p;
    return IDBF_OK;
  }
  template <typename T>
  idbf_status get(size_t n, T** out) {
    void* p = nullptr;
    idbf_status s = alloc(n * sizeof(T), &p);
    *out = static_cast<T*>(p);
    return s;
  }
  // chunks back to the cache once the device is idle
  void release() {
    if (!chunks.empty()) (void)hipDeviceSynchronize();
    for (auto& c : chunks) al.put(c.dev, c.base, c.size);
    chunks.clear();
    cur = nullptr;
    used = cap = total = 0;
  }
};

struct Batch {
  int side = 0, t = 0;
  int64_t n = 0;
  int32_t *cand_beg = nullptr, *cand_len = nullptr, *allow_beg = nullptr, *allow_len = nullptr;
  int32_t *samples = nullptr, *rank = nullptr, *skel_off = nullptr, *skel_idx = nullptr;
  double* skel_coord = nullptr;  // X (U side) or Omega (V side) of each skeleton index
  ApplyMeta* meta = nullptr;     // packed per-ID apply records
  int64_t *t_bound = nullptr, *T_off = nullptr;
  uint64_t* mask = nullptr;
  double2* T128 = nullptr;
  float2* T64 = nullptr;
  const int32_t* cand_arr = nullptr;
  const int32_t* allow_arr = nullptr;
  const double* cand_coord = nullptr;
  const double* allow_coord = nullptr;
  int64_t n_skel = 0, n_T = 0;   // n_T: reserved T entries (per-ID bounds, rounded even)
  int64_t nnz_T = 0;              // T entries in use: sum k (c - k)
  int64_t tb_max = 0;             // largest per-ID T reservation
  double flops = 0.0;             // FP64 flops of the batch's IDs
  int64_t sampled = 0;            // kernel entries sampled
  int rank_min = 0, rank_max = 0, cand_max = 0, s_max = 0;
  // learned proposal
  int32_t* s_prop = nullptr;   // sample counts the IDs used (proposal, or plain when rejected)
  int32_t* s_first = nullptr;  // the proposed counts, before the residual test
  float* y_rank = nullptr;     // the rank network's outputs (rank / 16)
  int32_t* prop_k = nullptr;     // skeleton proposal: number of proposed columns ...
  uint8_t* prop_cols = nullptr;  // ... and their positions, kMaxRank per ID
  int32_t* reject = nullptr;   // 1: proposal rejected by the residual test
  int64_t rejected = 0;
  int64_t tall = 0;               // IDs row-reduced before their QR (first pass)
  double wall_ms = 0.0;           // host wall time of the level
  std::chrono::steady_clock::time_point t0;
};

// HIP events around kernel launches, aggregated by name on request.
struct Profiler {
  struct Rec {
    const char* name;
    hipEvent_t a, b;
    double bytes, flops;
    bool a_shared;  // a is the end event of the record before (not owned)
  };
  bool on = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;

  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
  // returns a record index, or -1 when profiling is off
  int begin(const char* name, hipStream_t st) {
    if (!on) return -1;
    Rec r{name, event(), event(), 0.0, 0.0, false};
    if (!r.a || !r.b) return -1;
    (void)hipEventRecord(r.a, st);
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  // A record whose launch follows record prev's on the same stream with
  // nothing enqueued between them: it starts at prev's end event, so a chain
  // of n launches records n + 1 events instead of 2n (each record costs the
  // stream a marker).  prev < 0 starts a chain.
  int begin_after(int prev, const char* name, hipStream_t st) {
    if (!on) return -1;
    if (prev < 0) return begin(name, st);
    Rec r{name, recs[prev].b, event(), 0.0, 0.0, true};
    if (!r.b) return -1;
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(int id, hipStream_t st, double bytes = 0.0, double flops = 0.0) {
    if (id < 0) return;
    (void)hipEventRecord(recs[id].b, st);
    recs[id].bytes = bytes;
    recs[id].flops = flops;
  }
  void clear() {
    for (auto& r : recs) {
      if (!r.a_shared) pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
  ~Profiler() {
    clear();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

PhaseDev to_dev(const idbf_phase& p) { return PhaseDev{p.kind, p.c0, p.a, p.freq, p.cdiv}; }

idbf_status check_phase(const idbf_phase* phase) {
  if (!phase) {
    set_error("phase is NULL");
    return IDBF_EINVAL;
  }
  if (phase->kind != IDBF_PHASE_DFT && phase->kind != IDBF_PHASE_FIO && phase->kind != IDBF_PHASE_J0) {
    set_error("unknown phase kind %d", phase->kind);
    return IDBF_EINVAL;
  }
  if (phase->kind == IDBF_PHASE_FIO &&
      (!(phase->cdiv != 0.0) || !std::isfinite(phase->cdiv) || !std::isfinite(phase->c0) ||
       !std::isfinite(phase->a) || !std::isfinite(phase->freq))) {
    set_error("FIO phase parameters must be finite with cdiv != 0");
    return IDBF_EINVAL;
  }
  return IDBF_OK;
}

// finite and strictly ascending; result in *bad (device int) as a count of violations
__global__ void check_points_kernel(const double* p, int64_t n, int32_t* bad) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = p[i];
  bool ok = __builtin_isfinite(v);
  if (i + 1 < n) ok = ok && (p[i + 1] > v);
  if (!ok) atomicAdd(bad, 1);
}

// Values read back by the host between the phases of a level, staged in
// pinned memory so that many handles can be driven in lockstep with one
// synchronization per phase.
struct HostStage {
  int64_t st[12];
  unsigned long long counts[kBucketSlots];
  unsigned long long cursors[kBucketSlots];
  int32_t bad[2];
  double ends[2][2];  // first and last point of X and of Omega
};

struct LevelJob {
  Batch b;
  IdArgs ia;
  const double* X = nullptr;
  const double* Om = nullptr;
  int side = 0, t = 0;
};

}  // namespace
}  // namespace idbf

using namespace idbf;

struct idbf_plan_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // handles whose workspaces the graph writes: each counts this plan in
  // live_plans until idbf_plan_destroy, which keeps their workspaces in place
  std::vector<struct idbf_handle_s*> handles;
  ~idbf_plan_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

struct idbf_mlp_s {
  int hidden = 0;
  int np = 0;
  float* P = nullptr;  // parameters (device)
  float* M = nullptr;  // Adam moments
  float* V = nullptr;
  int step = 0;
  ~idbf_mlp_s() {
    if (P) (void)hipFree(P);
    if (M) (void)hipFree(M);
    if (V) (void)hipFree(V);
  }
};

struct idbf_handle_s {
  int64_t N = 0;
  int leaf = 0, L = 0, H = 0, kmax = 0, oversample = 1;
  double tol = 0.0;
  PhaseDev ph{};
  Arena arena;
  int32_t* iota = nullptr;
  int32_t* scratch = nullptr;  // skeleton lists before compaction (64 per ID)
  int32_t* order = nullptr;    // IDs of the current level grouped by QR wavefronts
  int32_t* tall_list = nullptr;  // tall IDs (more than kQrRows samples) of the current level
  unsigned long long* bucket = nullptr;  // [0, kBucketSlots): bucket counts, then the fill cursors
  // per-level scratch, grown as levels need it: sample positions, then the
  // tall IDs' slots, reduced blocks and reduction work space
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  int64_t* stats = nullptr;    // 12 int64 read back after each scan ([8, 11): work of every ID pass)
  int64_t* scan_ws = nullptr;  // tile partials of the prefix scans (kScanWs int64)
  int32_t* status = nullptr;
  std::vector<Batch> U, V;
  int64_t nblk = 0, nnz_S = 0, nnz_S_res = 0, sblk_max = 0;
  int32_t *s_rbeg = nullptr, *s_rlen = nullptr, *s_cbeg = nullptr, *s_clen = nullptr;
  int64_t *s_size = nullptr, *S_off = nullptr;
  double2* S128 = nullptr;
  float2* S64 = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t max_skel = 0;
  double construct_ms = 0.0;
  hipStream_t stream = nullptr;
  Profiler prof;
  HostStage* pin = nullptr;    // pinned: values the schedule reads back between phases
  LevelJob job;                // the level batch being built
  int qr_rec = -1;             // profiler record of that batch's QR launches
  idbf_mlp_s* proposer = nullptr;  // rank proposal network (not owned), or null
  idbf_mlp_s* skel_proposer = nullptr;  // skeleton proposal network (not owned), or null
  int sampler = IDBF_SAMPLER_MOCKCHEB;
  int margin = 0;
  double accept = IDBF_DEFAULT_ACCEPT;  // acceptance factor of the residual test
  uint64_t seed = 0;
  int live_plans = 0;          // captured plans that hold this handle's workspace pointer
  bool force_reject = false;   // IDBF_FLAG_PROPOSER_FORCE_REJECT
  bool apply_fuse = false;     // many-RHS apply: fused two-stage groups where eligible
  int rhs_iter = 0;            // many-RHS apply: right-hand-side blocks per workgroup (0: kernel default)
  bool truncate = false;       // IDBF_FLAG_ALLOW_TRUNCATE

  ~idbf_handle_s() {
    if (pin || ws || tmp) (void)hipDeviceSynchronize();  // nothing in flight uses them once they are held
    if (pin) chunk_cache().put_pinned(pin, sizeof(HostStage));
    if (ws) arena.al.put(current_device(), ws, ws_bytes);
    if (tmp) arena.al.put(current_device(), tmp, tmp_bytes);
    arena.release();
  }
};

namespace {

#define TRY(x)                          \
  do {                                  \
    idbf_status s_ = (x);               \
    if (s_ != IDBF_OK) return s_;       \
  } while (0)
#define TRYHIP(x) IDBF_HIP_CHECK(x)

idbf_status sync(idbf_handle_s* h) {
  IDBF_HIP_CHECK(hipStreamSynchronize(h->stream));
  return IDBF_OK;
}

// Construction of one level batch (U_t or V_t) in three phases; the host
// reads the pinned staging area between them, after the handle's stream has
// been synchronized.
//   level_begin:  descriptors, segment scans, QR bucket counts
//   level_ids:    sample selection, pivoted-QR IDs, rank scan
//   level_finish: skeleton compaction, packed per-ID records
idbf_status level_begin(idbf_handle_s* h, const double* X, const double* Om, int side, int t) {
  LevelJob& J = h->job;
  J = LevelJob{};
  J.X = X;
  J.Om = Om;
  J.side = side;
  J.t = t;
  Batch& b = J.b;
  b.side = side;
  b.t = t;
  b.t0 = std::chrono::steady_clock::now();
  b.n = int64_t(2) << h->L;
  const int64_t n = b.n;
  Arena& A = h->arena;
  TRY(A.get(n, &b.cand_beg));
  TRY(A.get(n, &b.cand_len));
  TRY(A.get(n, &b.allow_beg));
  TRY(A.get(n, &b.allow_len));
  TRY(A.get(n, &b.samples));
  TRY(A.get(n, &b.rank));
  TRY(A.get(n + 1, &b.skel_off));
  TRY(A.get(n, &b.t_bound));
  TRY(A.get(n + 1, &b.T_off));
  TRY(A.get(2 * n, &b.mask));

  const Batch* prev = nullptr;   // same side, level t-1
  const Batch* other = nullptr;  // allowed points' batch
  if (t > 1) prev = (side == IDBF_SIDE_U) ? &h->U[t - 2] : &h->V[t - 2];
  if (side == IDBF_SIDE_U) {
    if (t > 1) other = &h->V[t - 2];
  } else {
    other = &h->U[t - 1];
  }
  b.cand_arr = prev ? prev->skel_idx : h->iota;
  b.allow_arr = other ? other->skel_idx : h->iota;
  // on the first level the index arrays are the identity, so coordinates are X / Omega
  b.cand_coord = prev ? prev->skel_coord : (side == IDBF_SIDE_U ? X : Om);
  b.allow_coord = other ? other->skel_coord : (side == IDBF_SIDE_U ? Om : X);

  DescArgs d{};
  d.side = side;
  d.t = t;
  d.L = h->L;
  d.leaf = h->leaf;
  d.N = h->N;
  d.n_ids = n;
  d.oversample = h->oversample;
  d.kmax = h->kmax;
  d.prev_skel_off = prev ? prev->skel_off : nullptr;
  d.allow_skel_off = other ? other->skel_off : nullptr;
  d.cand_beg = b.cand_beg;
  d.cand_len = b.cand_len;
  d.allow_beg = b.allow_beg;
  d.allow_len = b.allow_len;
  d.t_bound = b.t_bound;
  d.samples = b.samples;
  int pr = h->prof.begin("level_desc", h->stream);
  TRYHIP(launch_desc(d, h->stream));
  TRYHIP(launch_scan_i64(b.t_bound, n, b.T_off, b.cand_len, h->stats, h->scan_ws, h->stream));
  TRYHIP(launch_scan_i32(b.samples, n, b.skel_off, nullptr, h->stats + 4, h->scan_ws, h->stream));
  const int32_t* qr_samples = b.samples;
  if (h->proposer) {  // proposed sample counts from the network's rank estimates
    float *F = nullptr, *y = nullptr;
    TRY(A.get(n * kProposalInputs, &F));
    TRY(A.get(n, &y));
    b.y_rank = y;
    TRY(A.get(n, &b.s_prop));
    TRY(A.get(n, &b.s_first));
    TRY(A.get(n, &b.reject));
    TRYHIP(launch_features(n, h->L, t, side == IDBF_SIDE_U ? 0 : 1, h->ph, F, h->stream));
    TRYHIP(launch_mlp_forward(h->proposer->P, kProposalInputs, h->proposer->hidden, F, n, y, nullptr, nullptr,
                              h->stream));
    TRYHIP(launch_propose(y, b.samples, n, h->oversample, h->margin, b.s_prop, h->stream));
    TRYHIP(hipMemcpyAsync(b.s_first, b.s_prop, n * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
    qr_samples = b.s_prop;
  }
  TRYHIP(hipMemsetAsync(h->bucket, 0, kBucketSlots * sizeof(unsigned long long), h->stream));
  TRYHIP(launch_bucket_count(qr_samples, b.cand_len, nullptr, n, h->bucket, h->stream));
  h->prof.end(pr, h->stream);
  TRYHIP(hipMemcpyAsync(h->pin->counts, h->bucket, sizeof h->pin->counts, hipMemcpyDeviceToHost, h->stream));
  TRYHIP(hipMemcpyAsync(h->pin->st, h->stats, sizeof h->pin->st, hipMemcpyDeviceToHost, h->stream));
  return IDBF_OK;
}

idbf_status level_scan(idbf_handle_s* h);

// Scratch of a level's ID passes in the handle's growable buffer: sample
// positions (s_max per ID) and, for the n_tall tall IDs, their slots,
// reduced c x c blocks and the reduction's s x c work blocks (a bounded
// number of them; the reduction runs in chunks).
constexpr size_t kTallWorkBytes = size_t(1) << 30;

idbf_status grow_tmp(idbf_handle_s* h, size_t bytes) {
  if (bytes <= h->tmp_bytes) return IDBF_OK;
  if (h->tmp) {
    IDBF_HIP_CHECK(hipStreamSynchronize(h->stream));  // the previous level's passes are done with it
    h->arena.al.put(current_device(), h->tmp, h->tmp_bytes);
    h->tmp = nullptr;
    h->tmp_bytes = 0;
  }
  if (h->arena.limit && h->arena.total + bytes > h->arena.limit) {
    set_error("device memory cap of %zu bytes exceeded (%zu held, %zu requested for level scratch)",
              (size_t)h->arena.limit, h->arena.total, bytes);
    return IDBF_ENOMEM;
  }
  size_t got = bytes;
  hipError_t e = h->arena.al.get(bytes, SIZE_MAX, &h->tmp, &got);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->tmp = nullptr;
    set_error("level scratch of %zu bytes: %s", bytes, hipGetErrorString(e));
    return IDBF_ENOMEM;
  }
  h->tmp_bytes = got;
  return IDBF_OK;
}

idbf_status level_scratch(idbf_handle_s* h, IdArgs& ia, int64_t n, int s_max, int c_max, int64_t n_tall,
                          size_t extra = 0, void** extra_ptr = nullptr) {
  const int64_t ld = std::max(1, s_max);
  size_t bytes = ((size_t(n) * ld * 4 + 255) & ~size_t(255)) + ((extra + 255) & ~size_t(255));
  size_t chunk = 0, slot_b = 0, R_b = 0;
  if (n_tall > 0) {
    const size_t work_ld = size_t(s_max) * c_max;
    chunk = std::max<size_t>(1, std::min<size_t>(n_tall, kTallWorkBytes / (work_ld * 16)));
    slot_b = (size_t(n) * 4 + 255) & ~size_t(255);
    R_b = size_t(n_tall) * c_max * c_max * 16;
    bytes += slot_b + R_b + chunk * work_ld * 16;
  }
  TRY(grow_tmp(h, bytes));
  char* p = static_cast<char*>(h->tmp);
  if (extra_ptr) *extra_ptr = p;
  p += (extra + 255) & ~size_t(255);
  ia.samp_pos = reinterpret_cast<int32_t*>(p);
  ia.samp_ld = ld;
  p += (size_t(n) * ld * 4 + 255) & ~size_t(255);
  ia.n_tall = n_tall;
  ia.tall_list = h->tall_list;
  if (n_tall > 0) {
    ia.tall_slot = reinterpret_cast<int32_t*>(p);
    p += slot_b;
    ia.tall_R = reinterpret_cast<double2*>(p);
    ia.tall_ld2 = int64_t(c_max) * c_max;
    p += R_b;
    ia.tall_work = reinterpret_cast<double2*>(p);
    ia.tall_work_ld = int64_t(s_max) * c_max;
    ia.tall_chunk = (int64_t)chunk;
  }
  return IDBF_OK;
}

idbf_status level_ids(idbf_handle_s* h) {
  LevelJob& J = h->job;
  Batch& b = J.b;
  const int side = J.side, t = J.t;
  const int64_t n = b.n;
  Arena& A = h->arena;
  const int64_t* st = h->pin->st;
  b.n_T = st[0];
  b.tb_max = st[1];
  b.cand_max = (int)st[3];
  b.s_max = (int)st[5];
  if (b.cand_max > kMaxCand) {
    set_error("level %d %c: a candidate set has %d points (max %d); ranks grew past %d", t,
              side == IDBF_SIDE_U ? 'U' : 'V', b.cand_max, kMaxCand, kMaxCand / 2);
    return IDBF_EUNSUPPORTED;
  }
  if (b.s_max > kMaxSamples) {
    set_error("level %d %c: an ID samples %d points (t |cand|; max %d)", t, side == IDBF_SIDE_U ? 'U' : 'V',
              b.s_max, kMaxSamples);
    return IDBF_EUNSUPPORTED;
  }
  TRY(A.get(std::max<int64_t>(b.n_T, 1), &b.T128));
  TRY(A.get(std::max<int64_t>(b.n_T, 1), &b.T64));

  IdArgs& ia = J.ia;
  ia = IdArgs{};
  ia.ph = h->ph;
  ia.X = J.X;
  ia.Om = J.Om;
  ia.side = side;
  ia.n_ids = n;
  ia.cand_idx = b.cand_arr;
  ia.cand_beg = b.cand_beg;
  ia.cand_len = b.cand_len;
  ia.cand_coord = b.cand_coord;
  ia.allow_idx = b.allow_arr;
  ia.allow_beg = b.allow_beg;
  ia.allow_len = b.allow_len;
  ia.allow_coord = b.allow_coord;
  ia.tol = h->tol;
  ia.kmax = h->kmax;
  ia.truncate = h->truncate;
  ia.oversample = h->oversample;
  ia.s_max = b.s_max;
  ia.c_max = b.cand_max;
  ia.sampler = h->sampler;
  ia.level = t;
  ia.seed = h->seed;
  b.tall = (int64_t)h->pin->counts[kQrBuckets];
  // skeleton proposal: candidate features and scores in the level scratch
  const size_t sk_bytes = h->skel_proposer ? size_t(n) * b.cand_max * (kProposalInputs + 1) * sizeof(float) : 0;
  void* sk = nullptr;
  TRY(level_scratch(h, ia, n, b.s_max, b.cand_max, b.tall, sk_bytes, &sk));
  if (h->skel_proposer) {
    float* F = static_cast<float*>(sk);
    float* score = F + size_t(n) * b.cand_max * kProposalInputs;
    TRY(A.get(n, &b.prop_k));
    TRY(A.get(n * kMaxRank, &b.prop_cols));
    const int pr = h->prof.begin("skel_propose", h->stream);
    TRYHIP(launch_cand_features(n, h->L, t, side == IDBF_SIDE_U ? 0 : 1, h->ph, b.cand_beg, b.cand_len,
                                b.cand_coord, b.cand_max, F, h->stream));
    TRYHIP(launch_mlp_forward(h->skel_proposer->P, kProposalInputs, h->skel_proposer->hidden, F,
                              n * b.cand_max, score, nullptr, nullptr, h->stream));
    TRYHIP(launch_pick_skeletons(score, b.cand_max, b.y_rank, b.s_prop, b.cand_len, n, h->margin, b.prop_k,
                                 b.prop_cols, h->stream));
    h->prof.end(pr, h->stream);
    ia.prop_k = b.prop_k;
    ia.prop_cols = b.prop_cols;
    ia.prop_fail = b.reject;  // read back by the residual test
    TRYHIP(hipMemsetAsync(b.reject, 0, size_t(n) * sizeof(int32_t), h->stream));
  }
  ia.order = h->order;
  ia.bucket_off[0] = 0;
  for (int w = 0; w < kQrBuckets; ++w) ia.bucket_off[w + 1] = ia.bucket_off[w] + (int64_t)h->pin->counts[w];
  for (int w = 0; w < kQrBuckets; ++w) h->pin->cursors[w] = (unsigned long long)ia.bucket_off[w];
  h->pin->cursors[kQrBuckets] = 0;
  TRYHIP(hipMemcpyAsync(h->bucket + kBucketSlots, h->pin->cursors, sizeof h->pin->cursors, hipMemcpyHostToDevice,
                        h->stream));
  ia.samples = b.s_prop;  // null without a proposer
  TRYHIP(launch_bucket_fill(b.s_prop ? b.s_prop : b.samples, b.cand_len, nullptr, n, h->bucket + kBucketSlots,
                            h->order, h->tall_list, h->stream));
  ia.rank = b.rank;
  ia.mask = b.mask;
  ia.skel_out = h->scratch;
  ia.T128 = b.T128;
  ia.T64 = b.T64;
  ia.T_off = b.T_off;
  ia.status = h->status;
  int pr = h->prof.begin("id_select", h->stream);
  TRYHIP(launch_select(ia, h->stream));
  h->prof.end(pr, h->stream);
  const int pq = h->prof.begin("id_qr", h->stream);
  TRYHIP(launch_qr(ia, h->stream));
  h->prof.end(pq, h->stream);
  h->qr_rec = pq;  // its flop count is attached once the work counters are back
  if (h->proposer) {  // residual test; rejected IDs are counted per QR bucket for the fallback
    TRYHIP(hipMemsetAsync(h->stats + 8, 0, 3 * sizeof(int64_t), h->stream));
    TRYHIP(launch_id_work(b.rank, b.cand_len, b.s_prop, nullptr, n, reinterpret_cast<unsigned long long*>(h->stats + 8),
                          h->stream));
    ResidualArgs ra{};
    ra.id = ia;
    ra.level = t;
    ra.seed = h->seed;
    ra.factor = h->accept;
    ra.force_reject = h->force_reject;
    ra.skeletons = h->skel_proposer != nullptr;
    ra.reject = b.reject;
    ra.s_prop = b.s_prop;
    ra.samples_plain = b.samples;
    pr = h->prof.begin("id_residual", h->stream);
    TRYHIP(launch_residual(ra, h->stream));
    h->prof.end(pr, h->stream);
    TRYHIP(hipMemsetAsync(h->bucket, 0, kBucketSlots * sizeof(unsigned long long), h->stream));
    TRYHIP(launch_bucket_count(b.s_prop, b.cand_len, b.reject, n, h->bucket, h->stream));
    TRYHIP(hipMemcpyAsync(h->pin->counts, h->bucket, sizeof h->pin->counts, hipMemcpyDeviceToHost, h->stream));
    return IDBF_OK;
  }
  return level_scan(h);
}

// Recompute the rejected proposals from the plain sample counts.
idbf_status level_fallback(idbf_handle_s* h) {
  LevelJob& J = h->job;
  Batch& b = J.b;
  IdArgs ia = J.ia;
  ia.prop_k = nullptr;  // the fallback is the plain pivoted ID
  ia.prop_cols = nullptr;
  ia.prop_fail = nullptr;
  ia.bucket_off[0] = 0;
  for (int w = 0; w < kQrBuckets; ++w) ia.bucket_off[w + 1] = ia.bucket_off[w] + (int64_t)h->pin->counts[w];
  b.rejected = ia.bucket_off[kQrBuckets];
  if (b.rejected > 0) {
    // scratch of this pass: sample positions and the rejected tall IDs' blocks
    TRY(level_scratch(h, ia, b.n, b.s_max, b.cand_max, (int64_t)h->pin->counts[kQrBuckets]));
    for (int w = 0; w < kQrBuckets; ++w) h->pin->cursors[w] = (unsigned long long)ia.bucket_off[w];
    h->pin->cursors[kQrBuckets] = 0;
    TRYHIP(hipMemcpyAsync(h->bucket + kBucketSlots, h->pin->cursors, sizeof h->pin->cursors, hipMemcpyHostToDevice,
                          h->stream));
    TRYHIP(launch_bucket_fill(b.s_prop, b.cand_len, b.reject, b.n, h->bucket + kBucketSlots, h->order,
                              h->tall_list, h->stream));
    ia.samples = b.s_prop;  // plain counts for the rejected IDs
    ia.sel_list = h->order;
    ia.sel_n = b.rejected;
    int pr = h->prof.begin("id_select", h->stream);
    TRYHIP(launch_select(ia, h->stream));
    h->prof.end(pr, h->stream);
    ia.sel_list = nullptr;
    pr = h->prof.begin("id_qr_fallback", h->stream);
    TRYHIP(launch_qr(ia, h->stream));
    h->prof.end(pr, h->stream);
    TRYHIP(launch_id_work(b.rank, b.cand_len, b.s_prop, b.reject, b.n,
                          reinterpret_cast<unsigned long long*>(h->stats + 8), h->stream));
  }
  return level_scan(h);
}

// Work counters and the rank scan of a finished batch, read back by level_finish.
idbf_status level_scan(idbf_handle_s* h) {
  LevelJob& J = h->job;
  Batch& b = J.b;
  const int64_t n = b.n;
  const int pr = h->prof.begin("level_scan", h->stream);
  TRYHIP(hipMemsetAsync(h->stats + 4, 0, 3 * sizeof(int64_t), h->stream));
  TRYHIP(launch_id_work(b.rank, b.cand_len, b.s_prop ? b.s_prop : b.samples, nullptr, n,
                        reinterpret_cast<unsigned long long*>(h->stats + 4), h->stream));
  TRYHIP(launch_scan_i32(b.rank, n, b.skel_off, nullptr, h->stats, h->scan_ws, h->stream));
  TRYHIP(hipMemcpyAsync(h->stats + 7, h->status, sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
  h->prof.end(pr, h->stream);
  TRYHIP(hipMemcpyAsync(h->pin->st, h->stats, sizeof h->pin->st, hipMemcpyDeviceToHost, h->stream));
  return IDBF_OK;
}

idbf_status level_finish(idbf_handle_s* h) {
  LevelJob& J = h->job;
  Batch& b = J.b;
  const int side = J.side, t = J.t;
  const int64_t n = b.n;
  Arena& A = h->arena;
  const int64_t* st = h->pin->st;
  b.flops = (double)(unsigned long long)st[4];
  b.nnz_T = st[5];
  b.sampled = st[6];
  if (h->proposer) {  // work of every pass: the proposals, then the recomputed rejections
    b.flops = (double)(unsigned long long)st[8];
    b.sampled = st[10];
  }
  if (h->qr_rec >= 0) h->prof.recs[h->qr_rec].flops = b.flops;
  const int32_t status = (int32_t)(st[7] & 0xffffffff);
  if (status & kErrRank) {
    set_error("level %d %c: an ID needs rank > %d at tol %g", t, side == IDBF_SIDE_U ? 'U' : 'V', kMaxRank,
              h->tol);
    return IDBF_ERANK;
  }
  if (status & kErrSize) {
    set_error("level %d %c: an ID exceeded the kernel's size limits", t, side == IDBF_SIDE_U ? 'U' : 'V');
    return IDBF_EUNSUPPORTED;
  }
  b.n_skel = st[0];
  b.rank_max = (int)st[1];
  b.rank_min = (int)st[2];
  TRY(A.get(std::max<int64_t>(b.n_skel, 1), &b.skel_idx));
  TRY(A.get(std::max<int64_t>(b.n_skel, 1), &b.skel_coord));
  TRY(A.get(n, &b.meta));
  const int pr = h->prof.begin("level_compact", h->stream);
  TRYHIP(launch_compact_skel(h->scratch, b.rank, b.skel_off, n, side == IDBF_SIDE_U ? J.X : J.Om, b.skel_idx,
                             b.skel_coord, h->stream));
  TRYHIP(launch_pack_meta(b.T_off, b.mask, b.cand_beg, b.skel_off, b.cand_len, b.rank, n, b.meta, h->stream));
  h->prof.end(pr, h->stream);
  h->max_skel = std::max(h->max_skel, b.n_skel);
  b.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - b.t0).count();
  if (side == IDBF_SIDE_U) h->U.push_back(b); else h->V.push_back(b);
  return IDBF_OK;
}

// Middle factor: block descriptors and sizes (phase 1), then the sampled
// blocks (phase 2).
idbf_status middle_begin(idbf_handle_s* h) {
  Arena& A = h->arena;
  if (h->H == 0) {
    h->nblk = 1;
    TRY(A.get(1, &h->s_rbeg));
    TRY(A.get(1, &h->s_rlen));
    TRY(A.get(1, &h->s_cbeg));
    TRY(A.get(1, &h->s_clen));
    TRY(A.get(2, &h->S_off));
    const int32_t zero = 0, nn = (int32_t)h->N;
    h->nnz_S = h->N * h->N;
    h->nnz_S_res = (h->nnz_S + 1) & ~int64_t(1);
    h->sblk_max = h->nnz_S_res;
    const int64_t offs[2] = {0, h->nnz_S_res};
    TRYHIP(hipMemcpyAsync(h->s_rbeg, &zero, 4, hipMemcpyHostToDevice, h->stream));
    TRYHIP(hipMemcpyAsync(h->s_cbeg, &zero, 4, hipMemcpyHostToDevice, h->stream));
    TRYHIP(hipMemcpyAsync(h->s_rlen, &nn, 4, hipMemcpyHostToDevice, h->stream));
    TRYHIP(hipMemcpyAsync(h->s_clen, &nn, 4, hipMemcpyHostToDevice, h->stream));
    TRYHIP(hipMemcpyAsync(h->S_off, offs, 16, hipMemcpyHostToDevice, h->stream));
    TRY(sync(h));  // the sources above live on this stack frame
    return IDBF_OK;
  }
  const int d = h->L - h->H + 1;
  h->nblk = int64_t(1) << (2 * d);
  TRY(A.get(h->nblk, &h->s_rbeg));
  TRY(A.get(h->nblk, &h->s_rlen));
  TRY(A.get(h->nblk, &h->s_cbeg));
  TRY(A.get(h->nblk, &h->s_clen));
  TRY(A.get(h->nblk, &h->s_size));
  TRY(A.get(h->nblk + 1, &h->S_off));
  MiddleDescArgs m{};
  m.L = h->L;
  m.H = h->H;
  m.n_blocks = h->nblk;
  m.u_off = h->U[h->H - 1].skel_off;
  m.v_off = h->V[h->H - 1].skel_off;
  m.rbeg = h->s_rbeg;
  m.rlen = h->s_rlen;
  m.cbeg = h->s_cbeg;
  m.clen = h->s_clen;
  m.size = h->s_size;
  m.nnz = reinterpret_cast<unsigned long long*>(h->stats + 4);
  TRYHIP(hipMemsetAsync(h->stats + 4, 0, sizeof(int64_t), h->stream));
  TRYHIP(launch_middle_desc(m, h->stream));
  TRYHIP(launch_scan_i64(h->s_size, h->nblk, h->S_off, nullptr, h->stats, h->scan_ws, h->stream));
  TRYHIP(hipMemcpyAsync(h->pin->st, h->stats, sizeof h->pin->st, hipMemcpyDeviceToHost, h->stream));
  return IDBF_OK;
}

idbf_status middle_finish(idbf_handle_s* h, const double* X, const double* Om) {
  Arena& A = h->arena;
  const int32_t* row_idx;
  const int32_t* col_idx;
  if (h->H == 0) {
    row_idx = col_idx = h->iota;
  } else {
    h->nnz_S_res = h->pin->st[0];
    h->sblk_max = h->pin->st[1];
    h->nnz_S = h->pin->st[4];
    row_idx = h->U[h->H - 1].skel_idx;
    col_idx = h->V[h->H - 1].skel_idx;
  }
  TRY(A.get(std::max<int64_t>(h->nnz_S_res, 1), &h->S128));
  TRY(A.get(std::max<int64_t>(h->nnz_S_res, 1), &h->S64));
  SampleBlocksArgs sb{};
  sb.ph = h->ph;
  sb.X = X;
  sb.Om = Om;
  sb.n_blocks = h->nblk;
  sb.row_idx = row_idx;
  sb.col_idx = col_idx;
  sb.rbeg = h->s_rbeg;
  sb.rlen = h->s_rlen;
  sb.cbeg = h->s_cbeg;
  sb.clen = h->s_clen;
  sb.off = h->S_off;
  sb.out128 = h->S128;
  sb.out64 = h->S64;
  const int pr = h->prof.begin("middle_sample", h->stream);
  TRYHIP(launch_sample_blocks(sb, h->stream));
  h->prof.end(pr, h->stream);
  return IDBF_OK;
}

// Input checks (finite, strictly ascending X and Omega): launch, then read.
idbf_status points_begin(idbf_handle_s* h, const double* X, const double* Om) {
  const double* pts[2] = {X, Om};
  for (int i = 0; i < 2; ++i) {
    TRYHIP(hipMemsetAsync(h->status, 0, sizeof(int32_t), h->stream));
    hipLaunchKernelGGL(check_points_kernel, dim3((unsigned)((h->N + 255) / 256)), dim3(256), 0, h->stream, pts[i],
                       h->N, h->status);
    TRYHIP(hipGetLastError());
    TRYHIP(hipMemcpyAsync(&h->pin->bad[i], h->status, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    TRYHIP(hipMemcpyAsync(&h->pin->ends[i][0], pts[i], sizeof(double), hipMemcpyDeviceToHost, h->stream));
    TRYHIP(hipMemcpyAsync(&h->pin->ends[i][1], pts[i] + (h->N - 1), sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
  }
  return IDBF_OK;
}

idbf_status points_finish(idbf_handle_s* h) {
  const char* names[2] = {"X", "Omega"};
  for (int i = 0; i < 2; ++i)
    if (h->pin->bad[i]) {
      set_error("%s must be finite and strictly ascending (%d violations)", names[i], h->pin->bad[i]);
      return IDBF_EINVAL;
    }
  if (h->ph.kind == IDBF_PHASE_J0) {
    // J_0's argument reduction is exact for |x xi| < 2^24 C1 (C1: pi/2 to 27 bits);
    // the points are ascending, so the largest |x| and |xi| sit at the ends
    const auto amax = [](const double* e) { return std::max(std::fabs(e[0]), std::fabs(e[1])); };
    const double zmax = amax(h->pin->ends[0]) * amax(h->pin->ends[1]);
    const double limit = 16777216.0 * 0x1.921fb54p0;
    if (!(zmax < limit)) {
      set_error("J0 kernel: max |x xi| = %g is beyond the supported %g", zmax, limit);
      return IDBF_EINVAL;
    }
  }
  return IDBF_OK;
}

// Device and pinned memory every construction needs before its first level.
idbf_status construct_setup(idbf_handle_s* h) {
  Arena& A = h->arena;
  if (!h->pin) {
    h->pin = static_cast<HostStage*>(chunk_cache().take_pinned(sizeof(HostStage)));
    if (!h->pin) {
      hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->pin), sizeof(HostStage), hipHostMallocDefault);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        h->pin = nullptr;
        set_error("pinned host allocation failed: %s", hipGetErrorString(e));
        return IDBF_ENOMEM;
      }
    }
    std::memset(h->pin, 0, sizeof(HostStage));
  }
  TRY(A.get(12, &h->stats));
  TRY(A.get(kScanWs, &h->scan_ws));
  TRY(A.get(1, &h->status));
  TRY(A.get(h->N, &h->iota));
  if (h->H > 0) {
    TRY(A.get((int64_t(2) << h->L) * kMaxCand, &h->scratch));
    TRY(A.get(int64_t(2) << h->L, &h->order));
    TRY(A.get(int64_t(2) << h->L, &h->tall_list));
    TRY(A.get(2 * kBucketSlots, &h->bucket));
  }
  return IDBF_OK;
}

idbf_status construct_start(idbf_handle_s* h, const double* X, const double* Om) {
  TRY(points_begin(h, X, Om));
  return IDBF_OK;
}

idbf_status construct_levels_ready(idbf_handle_s* h) {
  TRY(points_finish(h));
  TRYHIP(hipMemsetAsync(h->status, 0, sizeof(int32_t), h->stream));
  TRYHIP(launch_iota(h->iota, h->N, h->stream));
  return IDBF_OK;
}

idbf_status construct_impl(idbf_handle_s* h, const double* X, const double* Om) {
  TRY(construct_setup(h));
  TRY(construct_start(h, X, Om));
  TRY(sync(h));
  TRY(construct_levels_ready(h));
  for (int t = 1; t <= h->H; ++t)
    for (int side : {IDBF_SIDE_U, IDBF_SIDE_V}) {
      TRY(level_begin(h, X, Om, side, t));
      TRY(sync(h));
      TRY(level_ids(h));
      TRY(sync(h));
      if (h->proposer) {
        TRY(level_fallback(h));
        TRY(sync(h));
      }
      TRY(level_finish(h));
    }
  TRY(middle_begin(h));
  TRY(sync(h));
  TRY(middle_finish(h, X, Om));
  TRY(sync(h));
  return IDBF_OK;
}

idbf_status grow_workspace(idbf_handle_s* h, size_t bytes, hipStream_t st) {
  if (h->H == 0 || bytes <= h->ws_bytes) return IDBF_OK;
  if (h->live_plans > 0) {
    // a captured plan writes the current workspace: moving it would leave the
    // graph pointing at memory another handle may take over
    set_error("the apply workspace (%zu bytes) is held by %d captured plan(s); destroy them before applying "
              "with more right-hand sides (%zu bytes needed)",
              h->ws_bytes, h->live_plans, bytes);
    return IDBF_EINVAL;
  }
  if (h->ws) {
    (void)st;
    IDBF_HIP_CHECK(hipDeviceSynchronize());  // applies on any stream may still read it
    h->arena.al.put(current_device(), h->ws, h->ws_bytes);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t got = bytes;
  hipError_t e = h->arena.al.get(bytes, SIZE_MAX, &h->ws, &got);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->ws = nullptr;
    set_error("apply workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
    return IDBF_ENOMEM;
  }
  h->ws_bytes = got;
  return IDBF_OK;
}

const Batch* find_batch(const idbf_handle_s* h, int side, int level) {
  if (level < 1 || level > h->H) return nullptr;
  if (side == IDBF_SIDE_U) return &h->U[level - 1];
  if (side == IDBF_SIDE_V) return &h->V[level - 1];
  return nullptr;
}

}  // namespace

extern "C" {

void idbf_opts_default(idbf_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->oversample = 1;
}

const char* idbf_last_error(void) { return g_err; }

}  // extern "C"

namespace {

// Argument checks and an empty handle for one construction.
idbf_status make_handle(const idbf_phase* phase, const double* X, const double* Omega, int64_t N, double tol,
                        int32_t leaf, const idbf_opts& o, std::unique_ptr<idbf_handle_s>* out) {
  TRY(check_phase(phase));
  if (!X || !Omega) {
    set_error("X and Omega must be device pointers");
    return IDBF_EINVAL;
  }
  if (!is_pow2(leaf) || leaf > kMaxCand) {
    set_error("leaf must be a power of two in [1, %d], got %d", kMaxCand, leaf);
    return IDBF_EINVAL;
  }
  if (!is_pow2(N) || N < leaf || N > (int64_t(1) << 30)) {
    set_error("N must be a power of two in [leaf, 2^30], got %lld", (long long)N);
    return IDBF_EINVAL;
  }
  if (!(tol >= 0.0 && tol < 1.0)) {
    set_error("tol must satisfy 0 <= tol < 1, got %g", tol);
    return IDBF_EINVAL;
  }
  if (o.oversample < 1 || o.kmax < 0) {
    set_error("opts: oversample must be >= 1 and kmax >= 0");
    return IDBF_EINVAL;
  }
  std::unique_ptr<idbf_handle_s> h(new (std::nothrow) idbf_handle_s());
  if (!h) {
    set_error("host allocation failed");
    return IDBF_ENOMEM;
  }
  h->N = N;
  h->leaf = leaf;
  h->L = ilog2(N / leaf);
  h->H = h->L / 2;
  h->tol = tol;
  h->kmax = o.kmax;
  h->oversample = o.oversample;
  h->ph = to_dev(*phase);
  h->arena.limit = o.mem_cap_bytes;
  if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr)) {
    set_error("opts: dev_alloc and dev_free must be given together");
    return IDBF_EINVAL;
  }
  h->arena.al.alloc = o.dev_alloc;
  h->arena.al.free = o.dev_free;
  h->arena.al.user = o.alloc_user;
  h->arena.chunk_min = std::max<size_t>(size_t(64) << 20, size_t(N) * 2048);
  if (o.mem_cap_bytes) h->arena.chunk_min = std::min<size_t>(h->arena.chunk_min, o.mem_cap_bytes);
  h->stream = static_cast<hipStream_t>(o.stream);
  if (o.flags & ~(IDBF_FLAG_PROFILE | IDBF_FLAG_PROPOSER_FORCE_REJECT | IDBF_FLAG_ALLOW_TRUNCATE)) {
    set_error("opts: unknown flags 0x%x", (unsigned)o.flags);
    return IDBF_EINVAL;
  }
  h->prof.on = (o.flags & IDBF_FLAG_PROFILE) != 0;
  h->force_reject = (o.flags & IDBF_FLAG_PROPOSER_FORCE_REJECT) != 0;
  h->truncate = (o.flags & IDBF_FLAG_ALLOW_TRUNCATE) != 0;
  h->proposer = o.proposer;
  h->skel_proposer = o.skeleton_proposer;
  if (h->skel_proposer && !h->proposer) {
    set_error("opts: a skeleton proposer needs a rank proposer (opts.proposer)");
    return IDBF_EINVAL;
  }
  h->margin = o.proposal_margin;
  h->seed = o.seed;
  if (o.sampler != IDBF_SAMPLER_MOCKCHEB && o.sampler != IDBF_SAMPLER_RANDOM) {
    set_error("opts: unknown sampler %d", o.sampler);
    return IDBF_EINVAL;
  }
  h->sampler = o.sampler;
  if (h->proposer && o.proposal_margin < 0) {
    set_error("opts: proposal_margin must be >= 0");
    return IDBF_EINVAL;
  }
  if (!(o.proposal_accept >= 0.f) || !std::isfinite(o.proposal_accept)) {
    set_error("opts: proposal_accept must be finite and >= 0");
    return IDBF_EINVAL;
  }
  h->accept = o.proposal_accept > 0.f ? (double)o.proposal_accept : (double)IDBF_DEFAULT_ACCEPT;
  *out = std::move(h);
  return IDBF_OK;
}

void prefix_error(int i) {
  char msg[sizeof g_err];
  std::snprintf(msg, sizeof msg, "%s", g_err);
  set_error("instance %d: %s", i, msg);
}

constexpr int kBatchStreams = 4;  // hardware queues a process gets by default

// Device-lifetime streams for batched applies (default priority).
idbf_status pool_streams(std::vector<hipStream_t>* out) {
  static std::mutex mu;
  static std::vector<std::pair<int, std::vector<hipStream_t>>> pools;
  int dev = 0;
  IDBF_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  for (auto& p : pools)
    if (p.first == dev) {
      *out = p.second;
      return IDBF_OK;
    }
  std::vector<hipStream_t> s(kBatchStreams, nullptr);
  for (auto& x : s) IDBF_HIP_CHECK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
  pools.emplace_back(dev, s);
  *out = s;
  return IDBF_OK;
}

// caller stream -> every stream in `to` (fork) ...
idbf_status fork_streams(hipStream_t from, const std::vector<hipStream_t>& to) {
  hipEvent_t ev = nullptr;
  IDBF_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  hipError_t e = hipEventRecord(ev, from);
  for (size_t i = 0; e == hipSuccess && i < to.size(); ++i) e = hipStreamWaitEvent(to[i], ev, 0);
  (void)hipEventDestroy(ev);
  IDBF_HIP_CHECK(e);
  return IDBF_OK;
}

// ... and back (join)
idbf_status join_streams(const std::vector<hipStream_t>& from, hipStream_t to) {
  for (hipStream_t s : from) {
    hipEvent_t ev = nullptr;
    IDBF_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(to, ev, 0);
    (void)hipEventDestroy(ev);
    IDBF_HIP_CHECK(e);
  }
  return IDBF_OK;
}

idbf_status sync_streams(const std::vector<hipStream_t>& ss) {
  for (hipStream_t s : ss) IDBF_HIP_CHECK(hipStreamSynchronize(s));
  return IDBF_OK;
}

// Lockstep construction of several handles: every phase of every level is
// issued for all handles (each on one of `streams`), then the streams are
// synchronized once and the next phase reads the pinned staging areas.
idbf_status construct_lockstep(std::vector<std::unique_ptr<idbf_handle_s>>& hs, const double* const* X,
                               const double* const* Om, const std::vector<hipStream_t>& streams) {
  const int n = (int)hs.size();
#define IDBF_EACH(cond, call)                    \
  for (int i = 0; i < n; ++i) {                  \
    idbf_handle_s* h = hs[i].get();              \
    if (!(cond)) continue;                       \
    idbf_status s_ = (call);                     \
    if (s_ != IDBF_OK) {                         \
      prefix_error(i);                           \
      (void)sync_streams(streams);               \
      return s_;                                 \
    }                                            \
  }
  IDBF_EACH(true, construct_setup(h));
  IDBF_EACH(true, construct_start(h, X[i], Om[i]));
  TRY(sync_streams(streams));
  IDBF_EACH(true, construct_levels_ready(h));
  int Hmax = 0;
  for (auto& h : hs) Hmax = std::max(Hmax, h->H);
  for (int t = 1; t <= Hmax; ++t)
    for (int side : {IDBF_SIDE_U, IDBF_SIDE_V}) {
      IDBF_EACH(h->H >= t, level_begin(h, X[i], Om[i], side, t));
      TRY(sync_streams(streams));
      IDBF_EACH(h->H >= t, level_ids(h));
      TRY(sync_streams(streams));
      if (hs[0]->proposer) {  // every instance shares the options
        IDBF_EACH(h->H >= t, level_fallback(h));
        TRY(sync_streams(streams));
      }
      IDBF_EACH(h->H >= t, level_finish(h));
    }
  IDBF_EACH(true, middle_begin(h));
  TRY(sync_streams(streams));
  IDBF_EACH(true, middle_finish(h, X[i], Om[i]));
  TRY(sync_streams(streams));
#undef IDBF_EACH
  return IDBF_OK;
}

}  // namespace

extern "C" {

idbf_status idbf_construct(const idbf_phase* phase, const double* X, const double* Omega, int64_t N, double tol,
                           int32_t leaf, const idbf_opts* opts, idbf_handle* out) {
  g_err[0] = 0;
  if (!out) {
    set_error("out is NULL");
    return IDBF_EINVAL;
  }
  *out = nullptr;
  idbf_opts o;
  idbf_opts_default(&o);
  if (opts) o = *opts;
  auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<idbf_handle_s> h;
  TRY(make_handle(phase, X, Omega, N, tol, leaf, o, &h));
  idbf_status s = construct_impl(h.get(), X, Omega);
  if (s != IDBF_OK) {
    (void)hipStreamSynchronize(h->stream);
    return s;  // the handle's destructor frees everything
  }
  h->construct_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h.release();
  return IDBF_OK;
}

idbf_status idbf_construct_batched(int32_t count, const idbf_phase* phases, const double* const* X,
                                   const double* const* Omega, const int64_t* N, const double* tol,
                                   const int32_t* leaf, const idbf_opts* opts, idbf_handle* out) {
  g_err[0] = 0;
  if (count < 1 || !phases || !X || !Omega || !N || !tol || !leaf || !out) {
    set_error("construct_batched: count must be >= 1 and every array non-NULL");
    return IDBF_EINVAL;
  }
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  idbf_opts o;
  idbf_opts_default(&o);
  if (opts) o = *opts;
  auto t0 = std::chrono::steady_clock::now();
  std::vector<std::unique_ptr<idbf_handle_s>> hs(count);
  for (int i = 0; i < count; ++i) {
    idbf_status s = make_handle(&phases[i], X[i], Omega[i], N[i], tol[i], leaf[i], o, &hs[i]);
    if (s != IDBF_OK) {
      prefix_error(i);
      return s;
    }
  }
  std::vector<hipStream_t> streams;
  TRY(pool_streams(&streams));
  streams.resize(std::min<size_t>(streams.size(), (size_t)count));
  hipStream_t caller = static_cast<hipStream_t>(o.stream);
  TRY(fork_streams(caller, streams));  // X and Omega may come from work on the caller's stream
  for (int i = 0; i < count; ++i) hs[i]->stream = streams[i % streams.size()];
  idbf_status s = construct_lockstep(hs, X, Omega, streams);
  if (s != IDBF_OK) return s;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < count; ++i) {
    hs[i]->stream = caller;
    hs[i]->construct_ms = ms;
    out[i] = hs[i].release();
  }
  return IDBF_OK;
}

idbf_status idbf_destroy(idbf_handle h) {
  if (!h) return IDBF_OK;
  if (h->live_plans > 0) {
    set_error("destroy: %d captured plan(s) still use this handle; destroy them first", h->live_plans);
    return IDBF_EINVAL;
  }
  (void)hipDeviceSynchronize();
  delete h;
  return IDBF_OK;
}

idbf_status idbf_release_cached_memory(void) {
  chunk_cache().clear();
  return IDBF_OK;
}

idbf_status idbf_get_apply_config(idbf_handle h, idbf_apply_config* cfg) {
  g_err[0] = 0;
  if (!h || !cfg) {
    set_error("get_apply_config: NULL handle or config");
    return IDBF_EINVAL;
  }
  *cfg = idbf_apply_config{};
  cfg->fuse = h->apply_fuse ? 1 : 0;
  cfg->rhs_iter = h->rhs_iter;
  return IDBF_OK;
}

idbf_status idbf_set_apply_config(idbf_handle h, const idbf_apply_config* cfg) {
  g_err[0] = 0;
  if (!h || !cfg) {
    set_error("set_apply_config: NULL handle or config");
    return IDBF_EINVAL;
  }
  const int r = cfg->rhs_iter;
  if ((cfg->fuse != 0 && cfg->fuse != 1) || r < 0 || r > kMaxRhsIter || (r & (r - 1)) != 0) {
    set_error("set_apply_config: fuse must be 0 or 1 and rhs_iter 0 or a power of two <= %d", kMaxRhsIter);
    return IDBF_EINVAL;
  }
  h->apply_fuse = cfg->fuse == 1;
  h->rhs_iter = r;
  return IDBF_OK;
}

namespace {

// The stage arguments of level t of one side, shared by the apply and its
// adjoint.
StageArgs level_stage(const Batch& b, bool fp64, int64_t nrhs) {
  StageArgs a{};
  a.meta = b.meta;
  a.n = b.n;
  a.nrhs = nrhs;
  a.cand_beg = b.cand_beg;
  a.cand_len = b.cand_len;
  a.rank = b.rank;
  a.skel_off = b.skel_off;
  a.mask = b.mask;
  a.T_off = b.T_off;
  a.T = fp64 ? (const void*)b.T128 : (const void*)b.T64;
  a.pmax = (int)b.tb_max;
  a.cmax = b.cand_max;
  return a;
}

// y = K x (adj: y = K^H x, the stages in reverse order, each conjugate
// transposed).  Stage names of the profile: apply1_/applyn_/applyb_ (forward)
// or adj1_/adjn_/adjb_ (adjoint) + v, s, u.
// ws: the caller's workspace of ws_bytes (nothing allocated, nothing
// profiled), or null: the handle's own, grown as needed.
idbf_status apply_impl(idbf_handle h, const void* x, void* y, int64_t nrhs, int32_t dtype, void* stream, bool adj,
                       void* ws = nullptr, size_t ws_bytes = 0) {
  g_err[0] = 0;
  if (!h) {
    set_error("handle is NULL");
    return IDBF_EINVAL;
  }
  if (nrhs < 0 || (dtype != IDBF_C128 && dtype != IDBF_C64 && dtype != IDBF_C64_BF16X3)) {
    set_error("nrhs must be >= 0 and dtype IDBF_C128, IDBF_C64 or IDBF_C64_BF16X3");
    return IDBF_EINVAL;
  }
  if (nrhs == 0) return IDBF_OK;
  if (!x || !y || x == y) {
    set_error("x and y must be distinct device pointers");
    return IDBF_EINVAL;
  }
  const bool fp64 = dtype == IDBF_C128;
  const bool bf16 = dtype == IDBF_C64_BF16X3;
  // matrix-core stage kernels for more than one right-hand side (FP64 MFMA on
  // complex128, FP32 or BF16 split on complex64); a complex128 stage whose A
  // does not fit LDS runs on the VALU kernels
  const bool mfma = bf16 || nrhs > 1;
  const int prec = bf16 ? kGemmBf16 : fp64 ? kGemmF64 : kGemmF32;
  auto fits = [&](int kmax_unit, int mmax_unit) {
    return prec != kGemmF64 || gemm_lds_bytes(kmax_unit, mmax_unit, prec) <= kMaxGemmLds;
  };
  const size_t elem = fp64 ? 16 : 8;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t half = size_t(h->max_skel) * size_t(nrhs) * elem;
  const bool external = ws != nullptr;
  if (external) {
    if (2 * half > ws_bytes) {
      set_error("apply needs %zu bytes of workspace, %zu available", 2 * half, ws_bytes);
      return IDBF_EINVAL;
    }
  } else {
    TRY(grow_workspace(h, 2 * half, st));
    ws = h->ws;
  }
  // the caller's workspace path records no profile events (creating one may allocate)
  const bool prof_on = h->prof.on;
  struct ProfGuard {
    Profiler& p;
    bool keep;
    ~ProfGuard() { p.on = keep; }
  } guard{h->prof, prof_on};
  if (external) h->prof.on = false;
  char* buf[2] = {static_cast<char*>(ws), static_cast<char*>(ws) + half};
  int cur = 0;
  const void* in = x;
  // profile record names (the profiler keeps the pointer: literals only):
  // complex64 1 RHS, FP32 MFMA, BF16 split, complex128 1 RHS, complex128 many RHS
  static const char* const kNames[2][5][3] = {
      {{"apply1_v", "apply1_s", "apply1_u"}, {"applyn_v", "applyn_s", "applyn_u"},
       {"applyb_v", "applyb_s", "applyb_u"}, {"apply1d_v", "apply1d_s", "apply1d_u"},
       {"applynd_v", "applynd_s", "applynd_u"}},
      {{"adj1_v", "adj1_s", "adj1_u"}, {"adjn_v", "adjn_s", "adjn_u"}, {"adjb_v", "adjb_s", "adjb_u"},
       {"adj1d_v", "adj1d_s", "adj1d_u"}, {"adjnd_v", "adjnd_s", "adjnd_u"}}};
  const int kind = bf16 ? 2 : fp64 ? (nrhs == 1 ? 3 : 4) : (nrhs == 1 ? 0 : 1);
  auto name = [&](char stage) { return kNames[adj][kind][stage == 'v' ? 0 : stage == 's' ? 1 : 2]; };
  // one kernel launch per stage record, back to back on st: consecutive
  // records share their boundary event
  int prev = -1;
  auto rec_begin = [&](const char* nm) { return h->prof.begin_after(prev, nm, st); };
  auto rec_end = [&](int pr, double bytes, double flops) {
    h->prof.end(pr, st, bytes, flops);
    prev = pr;
  };
  // fused two-stage groups (complex64 FP32 MFMA, forward): the rank bound
  // of both levels picks the register tiles per part (0: not fusable)
  const bool fuse = h->apply_fuse && !adj && (prec == kGemmF32 || prec == kGemmBf16) && nrhs > 1;
  auto fuse_tk = [&](const Batch& b1, const Batch& b2, int kmax1, int mmax2) {
    const int r = std::max(b1.rank_max, b2.rank_max);
    const int tk = r <= 16 ? 1 : r <= 32 ? 2 : 0;
    if (!tk || kmax1 > 256 || mmax2 > 64 || fused2_lds_bytes(tk, kmax1, mmax2) > kMaxFusedLds) return 0;
    return tk;
  };
  // V-shaped stages: V_t forward (t = 1..H), U_t^H in the adjoint (t = 1..H)
  for (int t = 1; t <= h->H; ++t) {
    const Batch& b = adj ? h->U[t - 1] : h->V[t - 1];
    StageArgs a = level_stage(b, fp64, nrhs);
    a.rhs_iter = h->rhs_iter;
    a.in = in;
    a.out = buf[cur];
    if (fuse && t < h->H) {
      const Batch& b2 = h->V[t];
      const int tk = fuse_tk(b, b2, b.cand_max, 2 * b2.rank_max);
      if (tk) {
        a.n = b.n / 2;
        a.nn = 1 << (h->L - t + 1);
        StageArgs a2 = level_stage(b2, fp64, nrhs);
        a2.n = b2.n / 2;
        a2.nn = 1 << (h->L - t);
        a2.out = buf[cur];
        const double bytes = double(b.nnz_T + b2.nnz_T) * elem + 8.0 * (b.n + b2.n) +
                             (t == 1 ? double(h->N) * nrhs * elem : 0.0);
        const int pr = rec_begin(bf16 ? "applyb_vv" : "applyn_vv");
        IDBF_HIP_CHECK(launch_apply_fused2(a, a2, 0, tk, b.cand_max, 2 * b2.rank_max, prec, st));
        rec_end(pr, bytes, 8.0 * double(b.nnz_T + b2.nnz_T) * nrhs);
        in = buf[cur];
        cur ^= 1;
        ++t;
        continue;
      }
    }
    const double bytes = double(b.nnz_T) * elem + 8.0 * b.n + (t == 1 ? double(h->N) * nrhs * elem : 0.0);
    const int pr = rec_begin(name(adj ? 'u' : 'v'));
    if (mfma && fits(b.cand_max, 2 * b.rank_max)) {  // units: the ID pairs (C, 2P), (C, 2P + 1) sharing a segment
      StageArgs g = a;
      g.n = b.n / 2;
      g.nn = 1 << (h->L - t + 1);
      IDBF_HIP_CHECK(launch_apply_gemm(g, 0, b.cand_max, 2 * b.rank_max, prec, st, adj));
    } else {
      IDBF_HIP_CHECK(launch_apply_v(a, fp64, st, adj));
    }
    rec_end(pr, bytes, 8.0 * double(b.nnz_T) * nrhs);
    in = buf[cur];
    cur ^= 1;
  }
  {
    StageArgs a{};
    a.rhs_iter = h->rhs_iter;
    a.n = (h->H == 0) ? 1 : (adj ? h->V[h->H - 1].n : h->U[h->H - 1].n);
    a.nn = (h->H == 0) ? 1 : (1 << (h->L - h->H + 1));  // 2^d, used by the adjoint grouping
    a.nrhs = nrhs;
    a.nsub = (h->H == 0) ? 1 : (1 << (h->L - 2 * h->H + 1));
    a.rbeg = h->s_rbeg;
    a.rlen = h->s_rlen;
    a.cbeg = h->s_cbeg;
    a.clen = h->s_clen;
    a.T_off = h->S_off;
    a.T = fp64 ? (const void*)h->S128 : (const void*)h->S64;
    a.pmax = (int)h->sblk_max;
    a.dense = (h->H == 0);
    a.rlen_host = h->N;
    a.in = in;
    a.out = (h->H == 0) ? y : buf[cur];
    double bytes = double(h->nnz_S) * elem;
    if (h->H == 0) bytes += 2.0 * double(h->N) * nrhs * elem;
    const int pr = rec_begin(name('s'));
    const int kin = h->H == 0 ? 0 : adj ? h->U[h->H - 1].rank_max : h->V[h->H - 1].rank_max;
    const int mout = h->H == 0 ? 0 : adj ? h->V[h->H - 1].rank_max : h->U[h->H - 1].rank_max;
    if (mfma && !a.dense && fits(a.nsub * kin, mout)) {
      IDBF_HIP_CHECK(launch_apply_gemm(a, 1, a.nsub * kin, mout, prec, st, adj));
    } else {
      IDBF_HIP_CHECK(launch_apply_s(a, fp64, st, adj));
    }
    rec_end(pr, bytes, 8.0 * double(h->nnz_S) * nrhs);
    in = a.out;
    cur ^= 1;
  }
  // U-shaped stages: U_t forward (t = H..1), V_t^H in the adjoint (t = H..1)
  for (int t = h->H; t >= 1; --t) {
    const Batch& b = adj ? h->V[t - 1] : h->U[t - 1];
    StageArgs a = level_stage(b, fp64, nrhs);
    a.rhs_iter = h->rhs_iter;
    a.n = int64_t(1) << h->L;  // units: one per (node, parent partner)
    a.nn = 1 << (h->L - t + 1);
    a.in = in;
    a.out = (t == 1) ? y : buf[cur];
    if (fuse && t > 1) {
      const Batch& b2 = h->U[t - 2];
      const int tk = fuse_tk(b, b2, 2 * b.rank_max, b2.cand_max);
      if (tk) {
        StageArgs a2 = level_stage(b2, fp64, nrhs);
        a2.n = int64_t(1) << h->L;
        a2.nn = 1 << (h->L - t + 2);
        a2.out = (t == 2) ? y : buf[cur];
        const double bytes = double(b.nnz_T + b2.nnz_T) * elem + 8.0 * (b.n + b2.n) +
                             (t == 2 ? double(h->N) * nrhs * elem : 0.0);
        const int pr = rec_begin(bf16 ? "applyb_uu" : "applyn_uu");
        IDBF_HIP_CHECK(launch_apply_fused2(a, a2, 2, tk, 2 * b.rank_max, b2.cand_max, prec, st));
        rec_end(pr, bytes, 8.0 * double(b.nnz_T + b2.nnz_T) * nrhs);
        in = a2.out;
        cur ^= 1;
        --t;
        continue;
      }
    }
    const double bytes = double(b.nnz_T) * elem + 8.0 * b.n + (t == 1 ? double(h->N) * nrhs * elem : 0.0);
    const int pr = rec_begin(name(adj ? 'v' : 'u'));
    if (mfma && fits(2 * b.rank_max, b.cand_max))
      IDBF_HIP_CHECK(launch_apply_gemm(a, 2, 2 * b.rank_max, b.cand_max, prec, st, adj));
    else IDBF_HIP_CHECK(launch_apply_u(a, fp64, st, adj));
    rec_end(pr, bytes, 8.0 * double(b.nnz_T) * nrhs);
    in = a.out;
    cur ^= 1;
  }
  return IDBF_OK;
}

}  // namespace

idbf_status idbf_apply(idbf_handle h, const void* x, void* y, int64_t nrhs, int32_t dtype, void* stream) {
  return apply_impl(h, x, y, nrhs, dtype, stream, false);
}

idbf_status idbf_apply_adjoint(idbf_handle h, const void* x, void* y, int64_t nrhs, int32_t dtype, void* stream) {
  return apply_impl(h, x, y, nrhs, dtype, stream, true);
}

}  // extern "C"

namespace {

// The tuner's cache key: device, shape, the per-level rank and candidate
// bounds that decide every launch's tiles, right-hand sides and data type.
std::string tune_key(const idbf_handle_s* h, int64_t nrhs, int32_t dtype) {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    std::snprintf(prop.gcnArchName, sizeof prop.gcnArchName, "unknown");
  }
  std::string key = std::string(prop.gcnArchName) + " N=" + std::to_string(h->N) + " L=" + std::to_string(h->L) +
                    " H=" + std::to_string(h->H) + " nrhs=" + std::to_string(nrhs) + " dtype=" + std::to_string(dtype) +
                    " ranks=";
  for (int t = 0; t < h->H; ++t)
    key += std::to_string(h->V[t].rank_max) + "/" + std::to_string(h->V[t].cand_max) + "," +
           std::to_string(h->U[t].rank_max) + "/" + std::to_string(h->U[t].cand_max) + ";";
  for (char& ch : key)
    if (ch == '\t' || ch == '\n') ch = ' ';
  return key;
}

std::mutex& tune_file_mutex() {
  static std::mutex m;
  return m;
}

// Cache key of the QR-shape tuner: the device's architecture and the
// problem (phase parameters as exact hexadecimal floats).
std::string construct_key(const idbf_phase& p, int64_t N, double tol, int leaf, const idbf_opts& o) {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    std::snprintf(prop.gcnArchName, sizeof prop.gcnArchName, "unknown");
  }
  char buf[512];
  std::snprintf(buf, sizeof buf, "%s qr N=%lld phase=%d %a %a %a %a tol=%a leaf=%d t=%d kmax=%d sampler=%d",
                prop.gcnArchName, (long long)N, p.kind, p.c0, p.a, p.freq, p.cdiv, tol, leaf, o.oversample, o.kmax,
                o.sampler);
  std::string key(buf);
  for (char& ch : key)
    if (ch == '\t' || ch == '\n') ch = ' ';
  return key;
}

}  // namespace

extern "C" {

idbf_status idbf_tune_apply(idbf_handle h, int64_t nrhs, int32_t dtype, const char* cache_path, void* stream,
                            idbf_apply_config* chosen) {
  g_err[0] = 0;
  if (!h || nrhs < 1 || (dtype != IDBF_C128 && dtype != IDBF_C64 && dtype != IDBF_C64_BF16X3)) {
    set_error("tune_apply: NULL handle, nrhs < 1 or unknown dtype");
    return IDBF_EINVAL;
  }
  const std::string key = tune_key(h, nrhs, dtype);
  auto finish = [&](int fuse, int rhs_iter, float ms, bool cached) {
    h->apply_fuse = fuse == 1;
    h->rhs_iter = rhs_iter;
    if (chosen) {
      *chosen = idbf_apply_config{};
      chosen->fuse = fuse;
      chosen->rhs_iter = rhs_iter;
      chosen->from_cache = cached ? 1 : 0;
      chosen->ms = ms;
    }
    return IDBF_OK;
  };
  if (cache_path) {  // "<key>\t<fuse> <rhs_iter> <ms>" per line; the last line for a key wins
    std::lock_guard<std::mutex> lock(tune_file_mutex());
    if (FILE* f = std::fopen(cache_path, "r")) {
      std::vector<char> line(8192);
      int fuse = -1, rhs_iter = 0;
      float ms = 0.f;
      while (std::fgets(line.data(), (int)line.size(), f)) {
        char* tab = std::strchr(line.data(), '\t');
        if (!tab || std::string(line.data(), tab) != key) continue;
        int fz = 0, ri = 0;
        float m = 0.f;
        if (std::sscanf(tab + 1, "%d %d %f", &fz, &ri, &m) == 3 && (fz == 0 || fz == 1) && ri >= 0 &&
            ri <= kMaxRhsIter && (ri & (ri - 1)) == 0) {
          fuse = fz;
          rhs_iter = ri;
          ms = m;
        }
      }
      std::fclose(f);
      if (fuse >= 0) return finish(fuse, rhs_iter, ms, true);
    }
  }
  // time every candidate on scratch operands (an arbitrary finite pattern:
  // the kernels' timing does not depend on the values)
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t elem = dtype == IDBF_C128 ? 16 : 8;
  const size_t bytes = size_t(h->N) * size_t(nrhs) * elem;
  void *x = nullptr, *y = nullptr;
  if (hipMalloc(&x, bytes) != hipSuccess || hipMalloc(&y, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (x) (void)hipFree(x);
    set_error("tune_apply: cannot allocate %zu bytes of operands", 2 * bytes);
    return IDBF_ENOMEM;
  }
  struct Free {
    void *a, *b;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Free() {
      (void)hipFree(a);
      (void)hipFree(b);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } fr{x, y};
  IDBF_HIP_CHECK(hipMemsetAsync(x, 0x3c, bytes, st));
  IDBF_HIP_CHECK(hipEventCreate(&fr.e0));
  IDBF_HIP_CHECK(hipEventCreate(&fr.e1));
  const bool keep_fuse = h->apply_fuse;
  const int keep_iter = h->rhs_iter;
  const bool prof = h->prof.on;
  h->prof.on = false;
  const bool fusable = (dtype == IDBF_C64 || dtype == IDBF_C64_BF16X3) && nrhs > 1;
  const int64_t per_wave = dtype == IDBF_C128 ? 16 : dtype == IDBF_C64_BF16X3 ? 64 : 32;
  const int64_t blocks = (nrhs + 4 * per_wave - 1) / (4 * per_wave);  // right-hand-side blocks of 4 wavefronts
  int best_fuse = keep_fuse ? 1 : 0, best_iter = keep_iter;
  float best = -1.f;
  idbf_status s = IDBF_OK;
  const std::vector<int> fuses = fusable ? std::vector<int>{1, 0} : std::vector<int>{keep_fuse ? 1 : 0};
  for (const int fuse : fuses) {
    if (s != IDBF_OK) break;
    for (int r = 1; r <= 16 && s == IDBF_OK; r *= 2) {
      if (r > 1 && (r / 2) >= blocks) break;  // more blocks per workgroup than there are
      h->apply_fuse = fuse == 1;
      h->rhs_iter = r;
      s = apply_impl(h, x, y, nrhs, dtype, stream, false);  // warm-up (and workspace growth)
      if (s != IDBF_OK) break;
      if (hipEventRecord(fr.e0, st) != hipSuccess) s = IDBF_EHIP;
      for (int rep = 0; rep < 3 && s == IDBF_OK; ++rep) s = apply_impl(h, x, y, nrhs, dtype, stream, false);
      float ms = 0.f;
      if (s == IDBF_OK && (hipEventRecord(fr.e1, st) != hipSuccess || hipEventSynchronize(fr.e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, fr.e0, fr.e1) != hipSuccess)) {
        set_error("tune_apply: event timing failed");
        s = IDBF_EHIP;
      }
      if (s != IDBF_OK) break;
      ms /= 3.f;
      if (best < 0.f || ms < best) {
        best = ms;
        best_fuse = fuse;
        best_iter = r;
      }
    }
  }
  h->prof.on = prof;
  if (s != IDBF_OK) {
    h->apply_fuse = keep_fuse;
    h->rhs_iter = keep_iter;
    return s;
  }
  if (cache_path) {
    std::lock_guard<std::mutex> lock(tune_file_mutex());
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s\t%d %d %.4f\n", key.c_str(), best_fuse, best_iter, best);
      std::fclose(f);
    }
  }
  return finish(best_fuse, best_iter, best, false);
}

idbf_status idbf_set_qr_shapes(uint32_t mask) {
  g_err[0] = 0;
  if (mask & ~kQrShapeBits) {
    set_error("set_qr_shapes: mask 0x%x has bits above the three QR shape ranges", mask);
    return IDBF_EINVAL;
  }
  set_qr_shape_mask(mask);
  return IDBF_OK;
}

idbf_status idbf_get_qr_shapes(uint32_t* mask) {
  g_err[0] = 0;
  if (!mask) {
    set_error("get_qr_shapes: mask is NULL");
    return IDBF_EINVAL;
  }
  *mask = qr_shape_mask();
  return IDBF_OK;
}

idbf_status idbf_tune_construct(const idbf_phase* phase, const double* X, const double* Omega, int64_t N,
                                double tol, int32_t leaf, const idbf_opts* opts, const char* cache_path,
                                uint32_t* mask, float* ms, int32_t* from_cache) {
  g_err[0] = 0;
  TRY(check_phase(phase));
  if (!X || !Omega || N < 1) {
    set_error("tune_construct: X and Omega must be device arrays of N >= 1 points");
    return IDBF_EINVAL;
  }
  idbf_opts o;
  if (opts) o = *opts;
  else idbf_opts_default(&o);
  const std::string key = construct_key(*phase, N, tol, leaf, o);
  auto finish = [&](uint32_t m, float t, bool cached) {
    set_qr_shape_mask(m);
    if (mask) *mask = m;
    if (ms) *ms = t;
    if (from_cache) *from_cache = cached ? 1 : 0;
    return IDBF_OK;
  };
  if (cache_path) {  // "<key>\t<mask> <ms>" per line; the last line for a key wins
    std::lock_guard<std::mutex> lock(tune_file_mutex());
    if (FILE* f = std::fopen(cache_path, "r")) {
      std::vector<char> line(8192);
      long long found = -1;
      float t_found = 0.f;
      while (std::fgets(line.data(), (int)line.size(), f)) {
        char* tab = std::strchr(line.data(), '\t');
        if (!tab || std::string(line.data(), tab) != key) continue;
        unsigned m = 0;
        float t = 0.f;
        const int got = std::sscanf(tab + 1, "%u %f", &m, &t);
        if (got >= 1 && (m & ~kQrShapeBits) == 0) {
          found = m;
          t_found = got == 2 ? t : 0.f;
        }
      }
      std::fclose(f);
      if (found >= 0) return finish((uint32_t)found, t_found, true);
    }
  }
  o.flags |= IDBF_FLAG_PROFILE;
  const uint32_t keep = qr_shape_mask();
  // ID-kernel time of one construction with the shapes m (the better of two)
  auto time_shapes = [&](uint32_t m, int reps, float* out) -> idbf_status {
    set_qr_shape_mask(m);
    float best = -1.f;
    for (int rep = 0; rep < reps; ++rep) {
      idbf_handle h = nullptr;
      idbf_status s = idbf_construct(phase, X, Omega, N, tol, leaf, &o, &h);
      if (s != IDBF_OK) return s;
      idbf_kernel_stat st[64];
      int32_t n = 0;
      s = idbf_profile_read(h, st, 64, &n, 1);
      (void)idbf_destroy(h);
      if (s != IDBF_OK) return s;
      float t = 0.f;
      for (int i = 0; i < n; ++i)
        if (std::strncmp(st[i].name, "id_qr", 5) == 0) t += (float)st[i].ms;
      if (best < 0.f || t < best) best = t;
    }
    *out = best;
    return IDBF_OK;
  };
  float t_best = 0.f, t = 0.f;
  idbf_status s = time_shapes(keep, 1, &t);  // warm-up
  if (s == IDBF_OK) s = time_shapes(keep, 2, &t_best);
  uint32_t best = keep;
  for (uint32_t b = 0; b < 3 && s == IDBF_OK; ++b) {
    const uint32_t m = best ^ (1u << b);
    s = time_shapes(m, 2, &t);
    if (s == IDBF_OK && t < t_best) {
      best = m;
      t_best = t;
    }
  }
  if (s != IDBF_OK) {
    set_qr_shape_mask(keep);
    return s;
  }
  if (cache_path) {
    std::lock_guard<std::mutex> lock(tune_file_mutex());
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s\t%u %.4f\n", key.c_str(), best, t_best);
      std::fclose(f);
    }
  }
  return finish(best, t_best, false);
}

}  // extern "C"

// Device memory of idbf_apply_noalloc: one array per device, held until the
// process ends.  In host code the name is only a stand-in for the device
// array: its device address comes from hipGetSymbolAddress, once per device,
// and only that address is ever passed on.
static constexpr size_t kNoAllocBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

idbf_status noalloc_scratch(void** out) {
  static std::mutex mu;
  static int devs[64];
  static void* ptrs[64];
  static int n = 0;
  int dev = 0;
  IDBF_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  for (int i = 0; i < n; ++i)
    if (devs[i] == dev) {
      *out = ptrs[i];
      return IDBF_OK;
    }
  if (n == 64) {
    set_error("apply_noalloc: more than 64 devices");
    return IDBF_EUNSUPPORTED;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    set_error("apply_noalloc: hipGetSymbolAddress of the scratch array failed on device %d: %s", dev,
              hipGetErrorString(e));
    return IDBF_EHIP;
  }
  devs[n] = dev;
  ptrs[n] = ptr;
  ++n;
  *out = ptr;
  return IDBF_OK;
}

}  // namespace

extern "C" {

idbf_status idbf_apply_noalloc(idbf_handle h, const void* x, void* y, int64_t nrhs, int32_t dtype, void* stream) {
  g_err[0] = 0;
  if (!h) {
    set_error("handle is NULL");
    return IDBF_EINVAL;
  }
  if (nrhs > 0 && (dtype == IDBF_C128 || dtype == IDBF_C64 || dtype == IDBF_C64_BF16X3)) {
    const size_t need = 2 * size_t(h->max_skel) * size_t(nrhs) * (dtype == IDBF_C128 ? 16 : 8);
    if (h->H > 0 && need > kNoAllocBytes) {
      set_error("apply_noalloc: %lld right-hand sides need %zu bytes of workspace; the fixed scratch array "
                "holds %zu (use idbf_apply, or fewer right-hand sides)",
                (long long)nrhs, need, kNoAllocBytes);
      return IDBF_EINVAL;
    }
  }
  void* ws = nullptr;
  TRY(noalloc_scratch(&ws));
  return apply_impl(h, x, y, nrhs, dtype, stream, false, ws, kNoAllocBytes);
}

idbf_status idbf_apply_batched(int32_t count, const idbf_handle* hs, const void* const* x, void* const* y,
                               const int64_t* nrhs, int32_t dtype, void* stream) {
  g_err[0] = 0;
  if (count < 1 || !hs || !x || !y || !nrhs) {
    set_error("apply_batched: count must be >= 1 and every array non-NULL");
    return IDBF_EINVAL;
  }
  if (dtype != IDBF_C128 && dtype != IDBF_C64 && dtype != IDBF_C64_BF16X3) {
    set_error("apply_batched: unknown dtype %d", dtype);
    return IDBF_EINVAL;
  }
  std::vector<idbf_handle> sorted(hs, hs + count);
  std::sort(sorted.begin(), sorted.end());
  for (int i = 0; i < count; ++i)
    if (!sorted[i] || (i > 0 && sorted[i] == sorted[i - 1])) {
      set_error("apply_batched: handles must be non-NULL and distinct");
      return IDBF_EINVAL;
    }
  hipStream_t caller = static_cast<hipStream_t>(stream);
  const size_t elem = dtype == IDBF_C128 ? 16 : 8;
  for (int i = 0; i < count; ++i) {  // workspaces first: growing one synchronizes
    if (nrhs[i] < 0) {
      set_error("instance %d: nrhs must be >= 0", i);
      return IDBF_EINVAL;
    }
    idbf_status s = grow_workspace(hs[i], 2 * size_t(hs[i]->max_skel) * size_t(nrhs[i]) * elem, caller);
    if (s != IDBF_OK) {
      prefix_error(i);
      return s;
    }
  }
  std::vector<hipStream_t> streams;
  TRY(pool_streams(&streams));
  streams.resize(std::min<size_t>(streams.size(), (size_t)count));
  TRY(fork_streams(caller, streams));
  idbf_status st = IDBF_OK;
  for (int i = 0; i < count && st == IDBF_OK; ++i) {
    st = idbf_apply(hs[i], x[i], y[i], nrhs[i], dtype, streams[i % streams.size()]);
    if (st != IDBF_OK) prefix_error(i);
  }
  idbf_status sj = join_streams(streams, caller);  // joined even after a failure
  return st != IDBF_OK ? st : sj;
}

idbf_status idbf_apply_batched_plan(int32_t count, const idbf_handle* hs, const void* const* x, void* const* y,
                                    const int64_t* nrhs, int32_t dtype, void* stream, idbf_plan* out) {
  g_err[0] = 0;
  if (!out) {
    set_error("apply_batched_plan: out is NULL");
    return IDBF_EINVAL;
  }
  *out = nullptr;
  if (count < 1 || !hs || !x || !y || !nrhs) {
    set_error("apply_batched_plan: count must be >= 1 and every array non-NULL");
    return IDBF_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!st) {
    set_error("apply_batched_plan: a non-null stream is needed for capture");
    return IDBF_EINVAL;
  }
  // workspaces grow outside the capture (allocation is not capturable)
  const size_t elem = dtype == IDBF_C128 ? 16 : 8;
  for (int i = 0; i < count; ++i) {
    if (!hs[i] || nrhs[i] < 0) {
      set_error("apply_batched_plan: instance %d: NULL handle or negative nrhs", i);
      return IDBF_EINVAL;
    }
    idbf_status s = grow_workspace(hs[i], 2 * size_t(hs[i]->max_skel) * size_t(nrhs[i]) * elem, st);
    if (s != IDBF_OK) {
      prefix_error(i);
      return s;
    }
  }
  std::vector<hipStream_t> pool;
  TRY(pool_streams(&pool));  // created before the capture begins
  std::vector<bool> prof(count);
  for (int i = 0; i < count; ++i) {  // no event records inside the graph
    prof[i] = hs[i]->prof.on;
    hs[i]->prof.on = false;
  }
  std::unique_ptr<idbf_plan_s> plan(new (std::nothrow) idbf_plan_s());
  idbf_status s = IDBF_OK;
  if (!plan) {
    set_error("host allocation failed");
    s = IDBF_ENOMEM;
  }
  if (s == IDBF_OK) {
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("apply_batched_plan: hipStreamBeginCapture: %s", hipGetErrorString(e));
      s = IDBF_EHIP;
    } else {
      s = idbf_apply_batched(count, hs, x, y, nrhs, dtype, stream);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(st, &g);
      plan->graph = g;
      if (s == IDBF_OK && e != hipSuccess) {
        (void)hipGetLastError();
        set_error("apply_batched_plan: hipStreamEndCapture: %s", hipGetErrorString(e));
        s = IDBF_EHIP;
      }
      if (s == IDBF_OK) {
        e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          set_error("apply_batched_plan: hipGraphInstantiate: %s", hipGetErrorString(e));
          s = IDBF_EHIP;
        }
      }
    }
  }
  for (int i = 0; i < count; ++i) hs[i]->prof.on = prof[i];
  if (s != IDBF_OK) return s;
  plan->handles.assign(hs, hs + count);
  for (int i = 0; i < count; ++i) ++hs[i]->live_plans;
  *out = plan.release();
  return IDBF_OK;
}

idbf_status idbf_plan_launch(idbf_plan p, void* stream) {
  g_err[0] = 0;
  if (!p || !p->exec) {
    set_error("plan_launch: invalid plan");
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream)));
  return IDBF_OK;
}

idbf_status idbf_plan_destroy(idbf_plan p) {
  if (!p) return IDBF_OK;
  (void)hipDeviceSynchronize();
  for (idbf_handle_s* h : p->handles) --h->live_plans;
  delete p;
  return IDBF_OK;
}

idbf_status idbf_reserve(idbf_handle h, int64_t nrhs, int32_t dtype) {
  g_err[0] = 0;
  if (!h || nrhs < 0 || (dtype != IDBF_C128 && dtype != IDBF_C64 && dtype != IDBF_C64_BF16X3)) {
    set_error("reserve: invalid handle, nrhs or dtype");
    return IDBF_EINVAL;
  }
  const size_t elem = dtype == IDBF_C128 ? 16 : 8;
  return grow_workspace(h, 2 * size_t(h->max_skel) * size_t(nrhs) * elem, h->stream);
}

idbf_status idbf_get_info(idbf_handle h, idbf_info* info) {
  if (!h || !info) {
    set_error("handle and info must be non-NULL");
    return IDBF_EINVAL;
  }
  std::memset(info, 0, sizeof *info);
  info->N = h->N;
  info->leaf = h->leaf;
  info->L = h->L;
  info->H = h->H;
  info->oversample = h->oversample;
  info->tol = h->tol;
  info->nnz_S = h->nnz_S;
  info->rank_min = 1 << 30;
  for (const auto* side : {&h->U, &h->V}) {
    for (const Batch& b : *side) {
      info->n_ids += b.n;
      info->nnz_T += b.nnz_T;
      info->id_flops += b.flops;
      info->sampled_entries += b.sampled;
      info->n_skel += b.n_skel;
      info->rank_min = std::min(info->rank_min, b.rank_min);
      info->rank_max = std::max(info->rank_max, b.rank_max);
      info->cand_max = std::max(info->cand_max, b.cand_max);
      info->samples_max = std::max(info->samples_max, b.s_max);
      if (b.s_prop) info->proposed += b.n;
      info->rejected += b.rejected;
    }
  }
  if (info->n_ids == 0) info->rank_min = 0;
  info->device_bytes = (int64_t)(h->arena.total + h->ws_bytes + h->tmp_bytes);
  info->construct_ms = h->construct_ms;
  return IDBF_OK;
}

idbf_status idbf_stats(idbf_handle h, idbf_stats_t* out) {
  g_err[0] = 0;
  if (!h || !out) {
    set_error("stats: handle and out must be non-NULL");
    return IDBF_EINVAL;
  }
  std::memset(out, 0, sizeof *out);
  out->L = h->L;
  out->H = h->H;
  out->levels = std::min(h->H, IDBF_STATS_LEVELS);
  const int nb = 2 * out->levels;
  unsigned long long* hist = nullptr;
  std::vector<unsigned long long> hh(size_t(std::max(nb, 1)) * IDBF_STATS_RANKS, 0ull);
  if (nb > 0) {
    IDBF_HIP_CHECK(hipMalloc(&hist, hh.size() * sizeof(unsigned long long)));
    hipError_t e = hipMemsetAsync(hist, 0, hh.size() * sizeof(unsigned long long), h->stream);
    for (int t = 1; t <= out->levels && e == hipSuccess; ++t)
      for (int side = 0; side < 2 && e == hipSuccess; ++side) {
        const Batch& b = side == IDBF_SIDE_U ? h->U[t - 1] : h->V[t - 1];
        e = launch_rank_hist(b.rank, b.n, hist + size_t(2 * (t - 1) + side) * IDBF_STATS_RANKS, h->stream);
      }
    if (e == hipSuccess)
      e = hipMemcpyAsync(hh.data(), hist, hh.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    else (void)hipStreamSynchronize(h->stream);
    (void)hipFree(hist);
    if (e != hipSuccess) {
      set_error("stats: %s", hipGetErrorString(e));
      return IDBF_EHIP;
    }
  }
  int64_t records = 0, nnz_T = 0;
  for (int t = 1; t <= h->H; ++t)
    for (int side = 0; side < 2; ++side) {
      const Batch& b = side == IDBF_SIDE_U ? h->U[t - 1] : h->V[t - 1];
      records += b.n;
      nnz_T += b.nnz_T;
      if (t > out->levels) continue;
      idbf_level_stats_t& L = out->level[t - 1][side];
      L.n_ids = b.n;
      for (int r = 0; r < IDBF_STATS_RANKS; ++r) L.rank_hist[r] = (int64_t)hh[size_t(2 * (t - 1) + side) * IDBF_STATS_RANKS + r];
      L.rank_min = b.rank_min;
      L.rank_max = b.rank_max;
      L.cand_max = b.cand_max;
      L.samples_max = b.s_max;
      L.n_skel = b.n_skel;
      L.nnz_T = b.nnz_T;
      L.sampled_entries = b.sampled;
      L.tall = b.tall;
      L.proposed = b.s_prop ? b.n : 0;
      L.rejected = b.rejected;
      L.accepted = L.proposed - L.rejected;
      L.id_flops = b.flops;
      L.wall_ms = b.wall_ms;
    }
  out->nnz_S = h->nnz_S;
  out->n_blocks_S = h->nblk;
  out->apply_bytes_c64 = 8 * (nnz_T + h->nnz_S) + 40 * records;
  out->apply_bytes_c128 = 16 * (nnz_T + h->nnz_S) + 40 * records;
  out->device_bytes = (int64_t)(h->arena.total + h->ws_bytes + h->tmp_bytes);
  out->construct_ms = h->construct_ms;
  return IDBF_OK;
}

idbf_status idbf_profile_enable(idbf_handle h, int32_t on) {
  g_err[0] = 0;
  if (!h) {
    set_error("profile_enable: handle is NULL");
    return IDBF_EINVAL;
  }
  h->prof.on = on != 0;
  return IDBF_OK;
}

idbf_status idbf_profile_read(idbf_handle h, idbf_kernel_stat* out, int32_t max, int32_t* n, int32_t reset) {
  if (!h || !n || max < 0 || (max > 0 && !out)) {
    set_error("profile_read: handle, n and out must be valid");
    return IDBF_EINVAL;
  }
  if (!h->prof.on && h->prof.recs.empty()) {
    set_error("profiling is off for this handle (construct with IDBF_FLAG_PROFILE or call idbf_profile_enable)");
    return IDBF_EINVAL;
  }
  std::vector<idbf_kernel_stat> agg;
  for (auto& r : h->prof.recs) {
    IDBF_HIP_CHECK(hipEventSynchronize(r.b));
    float ms = 0.f;
    IDBF_HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
    idbf_kernel_stat* e = nullptr;
    for (auto& x : agg)
      if (std::strncmp(x.name, r.name, sizeof x.name) == 0) e = &x;
    if (!e) {
      agg.push_back(idbf_kernel_stat{});
      e = &agg.back();
      std::snprintf(e->name, sizeof e->name, "%s", r.name);
    }
    e->launches += 1;
    e->ms += ms;
    e->bytes += r.bytes;
    e->flops += r.flops;
  }
  const int m = std::min<int>(max, (int)agg.size());
  for (int i = 0; i < m; ++i) out[i] = agg[i];
  *n = m;
  if (reset) h->prof.clear();
  return IDBF_OK;
}

idbf_status idbf_batch_sizes(idbf_handle h, int32_t side, int32_t level, int64_t* n_ids, int64_t* n_skel,
                             int64_t* n_T) {
  if (!h) {
    set_error("handle is NULL");
    return IDBF_EINVAL;
  }
  const Batch* b = find_batch(h, side, level);
  if (!b) {
    set_error("no batch for side %d level %d (H = %d)", side, level, h->H);
    return IDBF_EINVAL;
  }
  if (n_ids) *n_ids = b->n;
  if (n_skel) *n_skel = b->n_skel;
  if (n_T) *n_T = b->n_T;
  return IDBF_OK;
}

idbf_status idbf_batch_export(idbf_handle h, int32_t side, int32_t level, int32_t* rank, int32_t* cand_len,
                              uint64_t* mask, int32_t* skel, double* T, int64_t* T_off) {
  if (!h) {
    set_error("handle is NULL");
    return IDBF_EINVAL;
  }
  const Batch* b = find_batch(h, side, level);
  if (!b) {
    set_error("no batch for side %d level %d (H = %d)", side, level, h->H);
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(hipDeviceSynchronize());
  if (rank) IDBF_HIP_CHECK(hipMemcpy(rank, b->rank, b->n * 4, hipMemcpyDeviceToHost));
  if (cand_len) IDBF_HIP_CHECK(hipMemcpy(cand_len, b->cand_len, b->n * 4, hipMemcpyDeviceToHost));
  if (mask) IDBF_HIP_CHECK(hipMemcpy(mask, b->mask, b->n * 16, hipMemcpyDeviceToHost));
  if (skel) IDBF_HIP_CHECK(hipMemcpy(skel, b->skel_idx, b->n_skel * 4, hipMemcpyDeviceToHost));
  if (T) IDBF_HIP_CHECK(hipMemcpy(T, b->T128, b->n_T * 16, hipMemcpyDeviceToHost));
  if (T_off) IDBF_HIP_CHECK(hipMemcpy(T_off, b->T_off, b->n * 8, hipMemcpyDeviceToHost));
  return IDBF_OK;
}

idbf_status idbf_batch_proposal(idbf_handle h, int32_t side, int32_t level, int32_t* proposed, int32_t* used,
                                int32_t* rejected) {
  g_err[0] = 0;
  const Batch* b = h ? find_batch(h, side, level) : nullptr;
  if (!b) {
    set_error("batch_proposal: invalid handle, side or level");
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(hipStreamSynchronize(h->stream));
  const size_t bytes = size_t(b->n) * sizeof(int32_t);
  const int32_t* first = b->s_first ? b->s_first : b->samples;
  const int32_t* final_ = b->s_prop ? b->s_prop : b->samples;
  if (proposed) IDBF_HIP_CHECK(hipMemcpy(proposed, first, bytes, hipMemcpyDeviceToHost));
  if (used) IDBF_HIP_CHECK(hipMemcpy(used, final_, bytes, hipMemcpyDeviceToHost));
  if (rejected) {
    if (b->reject) IDBF_HIP_CHECK(hipMemcpy(rejected, b->reject, bytes, hipMemcpyDeviceToHost));
    else std::memset(rejected, 0, bytes);
  }
  return IDBF_OK;
}

idbf_status idbf_batch_skeleton_proposal(idbf_handle h, int32_t side, int32_t level, int32_t* n_prop,
                                        uint8_t* order) {
  g_err[0] = 0;
  const Batch* b = h ? find_batch(h, side, level) : nullptr;
  if (!b || !b->prop_k) {
    set_error("batch_skeleton_proposal: invalid handle, side or level, or no skeleton proposer");
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(hipStreamSynchronize(h->stream));
  if (n_prop) IDBF_HIP_CHECK(hipMemcpy(n_prop, b->prop_k, size_t(b->n) * 4, hipMemcpyDeviceToHost));
  if (order) IDBF_HIP_CHECK(hipMemcpy(order, b->prop_cols, size_t(b->n) * kMaxRank, hipMemcpyDeviceToHost));
  return IDBF_OK;
}

idbf_status idbf_skeleton_samples(idbf_handle h, int32_t side, int32_t level, int32_t* cmax, float* features,
                                  float* targets) {
  g_err[0] = 0;
  const Batch* b = h ? find_batch(h, side, level) : nullptr;
  if (!b || !cmax) {
    set_error("skeleton_samples: invalid handle, side or level, or NULL cmax");
    return IDBF_EINVAL;
  }
  *cmax = b->cand_max;
  if (!features && !targets) return IDBF_OK;
  if (!features || !targets) {
    set_error("skeleton_samples: features and targets must both be given");
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(launch_cand_features(b->n, h->L, level, side == IDBF_SIDE_U ? 0 : 1, h->ph, b->cand_beg,
                                      b->cand_len, b->cand_coord, b->cand_max, features, h->stream));
  IDBF_HIP_CHECK(launch_skel_targets(b->mask, b->cand_len, b->n, b->cand_max, targets, h->stream));
  IDBF_HIP_CHECK(hipStreamSynchronize(h->stream));
  return IDBF_OK;
}

idbf_status idbf_middle_sizes(idbf_handle h, int64_t* n_blocks, int64_t* n_entries) {
  if (!h) {
    set_error("handle is NULL");
    return IDBF_EINVAL;
  }
  if (n_blocks) *n_blocks = h->nblk;
  if (n_entries) *n_entries = h->nnz_S_res;
  return IDBF_OK;
}

idbf_status idbf_middle_export(idbf_handle h, double* S, int64_t* S_off) {
  if (!h) {
    set_error("handle is NULL");
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(hipDeviceSynchronize());
  if (S) IDBF_HIP_CHECK(hipMemcpy(S, h->S128, h->nnz_S_res * 16, hipMemcpyDeviceToHost));
  if (S_off) IDBF_HIP_CHECK(hipMemcpy(S_off, h->S_off, h->nblk * 8, hipMemcpyDeviceToHost));
  return IDBF_OK;
}

idbf_status idbf_sample(const idbf_phase* phase, const double* X, const double* Omega, const int32_t* rows,
                        int64_t nrows, const int32_t* cols, int64_t ncols, double* out, void* stream) {
  g_err[0] = 0;
  TRY(check_phase(phase));
  if (nrows < 0 || ncols < 0) {
    set_error("nrows and ncols must be >= 0");
    return IDBF_EINVAL;
  }
  if (nrows * ncols == 0) return IDBF_OK;
  if (!X || !Omega || !rows || !cols || !out) {
    set_error("sampler pointers must be non-NULL");
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(launch_sample_dense(to_dev(*phase), X, Omega, rows, nrows, cols, ncols,
                                     reinterpret_cast<double2*>(out), static_cast<hipStream_t>(stream)));
  return IDBF_OK;
}

idbf_status idbf_id_batch(const idbf_phase* phase, const double* X, const double* Omega, int32_t side,
                          int64_t n_ids, const int32_t* cand_idx, const int32_t* cand_beg, const int32_t* cand_len,
                          const int32_t* allow_idx, const int32_t* allow_beg, const int32_t* allow_len, double tol,
                          int32_t kmax, int32_t oversample, int32_t* rank, uint64_t* mask, int32_t* skel, double* T,
                          void* stream) {
  g_err[0] = 0;
  TRY(check_phase(phase));
  if (side != IDBF_SIDE_U && side != IDBF_SIDE_V) {
    set_error("side must be IDBF_SIDE_U or IDBF_SIDE_V");
    return IDBF_EINVAL;
  }
  if (n_ids < 0 || oversample < 1 || kmax < 0 || !(tol >= 0.0 && tol < 1.0) || n_ids > INT32_MAX) {
    set_error("invalid n_ids, oversample, kmax or tol");
    return IDBF_EINVAL;
  }
  if (n_ids == 0) return IDBF_OK;
  if (!X || !Omega || !cand_idx || !cand_beg || !cand_len || !allow_idx || !allow_beg || !allow_len || !rank ||
      !mask || !skel || !T) {
    set_error("id_batch pointers must be non-NULL");
    return IDBF_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int32_t> cl(n_ids), al(n_ids);
  IDBF_HIP_CHECK(hipMemcpyAsync(cl.data(), cand_len, n_ids * 4, hipMemcpyDeviceToHost, st));
  IDBF_HIP_CHECK(hipMemcpyAsync(al.data(), allow_len, n_ids * 4, hipMemcpyDeviceToHost, st));
  IDBF_HIP_CHECK(hipStreamSynchronize(st));
  int smax = 0, cmax = 0, rows_max = 0;
  std::vector<int32_t> tall;
  for (int64_t q = 0; q < n_ids; ++q) {
    if (cl[q] < 1 || cl[q] > kMaxCand || al[q] < 1) {
      set_error("ID %lld: candidate count %d must be in [1, %d] and allowed count %d >= 1", (long long)q, cl[q],
                kMaxCand, al[q]);
      return IDBF_EINVAL;
    }
    const int64_t sq = std::min<int64_t>((int64_t)oversample * cl[q], al[q]);
    if (sq > kMaxSamples) {
      set_error("ID %lld samples %lld points (oversample x candidates; max %d)", (long long)q, (long long)sq,
                kMaxSamples);
      return IDBF_EUNSUPPORTED;
    }
    smax = std::max<int>(smax, (int)sq);
    cmax = std::max(cmax, cl[q]);
    rows_max = std::max(rows_max, qr_rows(cl[q], (int)sq));
    if (is_tall((int)sq)) tall.push_back((int32_t)q);
  }
  // one device block: status, sample positions, and the tall IDs' list,
  // slots, reduced blocks and reduction work space
  const int64_t n_tall = (int64_t)tall.size();
  const size_t work_ld = size_t(smax) * cmax;
  const size_t chunk = n_tall ? std::max<size_t>(1, std::min<size_t>(n_tall, kTallWorkBytes / (work_ld * 16))) : 0;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t b_pos = up(size_t(n_ids) * smax * 4), b_list = up(size_t(n_tall) * 4), b_slot = up(size_t(n_ids) * 4);
  const size_t b_R = size_t(n_tall) * cmax * cmax * 16, b_work = chunk * work_ld * 16;
  const size_t total = 256 + b_pos + (n_tall ? b_list + b_slot + b_R + b_work : 0);
  char* blk = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&blk), total) != hipSuccess) {
    (void)hipGetLastError();
    set_error("id_batch: no memory for %lld IDs' scratch (%zu bytes)", (long long)n_ids, total);
    return IDBF_ENOMEM;
  }
  int32_t* status = reinterpret_cast<int32_t*>(blk);
  IdArgs ia{};
  ia.samp_pos = reinterpret_cast<int32_t*>(blk + 256);
  ia.samp_ld = std::max(1, smax);
  hipError_t e = hipMemsetAsync(status, 0, sizeof(int32_t), st);
  if (n_tall) {
    char* p = blk + 256 + b_pos;
    int32_t* list = reinterpret_cast<int32_t*>(p);
    ia.tall_list = list;
    ia.n_tall = n_tall;
    ia.tall_slot = reinterpret_cast<int32_t*>(p + b_list);
    ia.tall_R = reinterpret_cast<double2*>(p + b_list + b_slot);
    ia.tall_ld2 = int64_t(cmax) * cmax;
    ia.tall_work = reinterpret_cast<double2*>(p + b_list + b_slot + b_R);
    ia.tall_work_ld = (int64_t)work_ld;
    ia.tall_chunk = (int64_t)chunk;
    if (e == hipSuccess) e = hipMemcpyAsync(list, tall.data(), size_t(n_tall) * 4, hipMemcpyHostToDevice, st);
  }
  ia.ph = to_dev(*phase);
  ia.X = X;
  ia.Om = Omega;
  ia.side = side;
  ia.n_ids = n_ids;
  ia.cand_idx = cand_idx;
  ia.cand_beg = cand_beg;
  ia.cand_len = cand_len;
  ia.allow_idx = allow_idx;
  ia.allow_beg = allow_beg;
  ia.allow_len = allow_len;
  ia.tol = tol;
  ia.kmax = kmax;
  ia.oversample = oversample;
  ia.s_max = smax;
  ia.c_max = cmax;
  ia.rows_max = rows_max;
  ia.rank = rank;
  ia.mask = mask;
  ia.skel_out = skel;
  ia.T128 = reinterpret_cast<double2*>(T);
  ia.T64 = nullptr;
  ia.T_off = nullptr;
  ia.status = status;
  if (e == hipSuccess) e = launch_id_batch(ia, st);
  int32_t flag = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&flag, status, sizeof flag, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  else (void)hipStreamSynchronize(st);  // nothing may still use the block when it is freed
  (void)hipFree(blk);
  if (e != hipSuccess) {
    set_error("id_batch: %s", hipGetErrorString(e));
    return IDBF_EHIP;
  }
  if (flag & kErrRank) {
    set_error("an ID needs rank > %d at tol %g", kMaxRank, tol);
    return IDBF_ERANK;
  }
  if (flag & kErrSize) {
    set_error("an ID exceeded the kernel's size limits");
    return IDBF_EUNSUPPORTED;
  }
  return IDBF_OK;
}

int32_t idbf_mlp_param_count(int32_t hidden) { return mlp_param_count(kProposalInputs, hidden); }

idbf_status idbf_mlp_create(int32_t hidden, const float* params, idbf_mlp* out) {
  g_err[0] = 0;
  if (!out || !params || (hidden != 16 && hidden != 32 && hidden != 64 && hidden != 128)) {
    set_error("mlp_create: hidden must be 16, 32, 64 or 128 and params/out non-NULL");
    return IDBF_EINVAL;
  }
  *out = nullptr;
  std::unique_ptr<idbf_mlp_s> m(new (std::nothrow) idbf_mlp_s());
  if (!m) {
    set_error("host allocation failed");
    return IDBF_ENOMEM;
  }
  m->hidden = hidden;
  m->np = mlp_param_count(kProposalInputs, hidden);
  const size_t bytes = size_t(m->np) * sizeof(float);
  for (float** p : {&m->P, &m->M, &m->V}) {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      set_error("mlp_create: hipMalloc failed");
      return IDBF_ENOMEM;
    }
  }
  IDBF_HIP_CHECK(hipMemcpy(m->P, params, bytes, hipMemcpyHostToDevice));
  IDBF_HIP_CHECK(hipMemset(m->M, 0, bytes));
  IDBF_HIP_CHECK(hipMemset(m->V, 0, bytes));
  *out = m.release();
  return IDBF_OK;
}

idbf_status idbf_mlp_destroy(idbf_mlp m) {
  if (!m) return IDBF_OK;
  (void)hipDeviceSynchronize();
  delete m;
  return IDBF_OK;
}

idbf_status idbf_mlp_params(idbf_mlp m, float* params) {
  if (!m || !params) {
    set_error("mlp_params: NULL argument");
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(hipMemcpy(params, m->P, size_t(m->np) * sizeof(float), hipMemcpyDeviceToHost));
  return IDBF_OK;
}

idbf_status idbf_mlp_forward(idbf_mlp m, const float* X, int64_t n, float* y, void* stream) {
  g_err[0] = 0;
  if (!m || n < 0 || (n > 0 && (!X || !y))) {
    set_error("mlp_forward: invalid arguments");
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(launch_mlp_forward(m->P, kProposalInputs, m->hidden, X, n, y, nullptr, nullptr,
                                    static_cast<hipStream_t>(stream)));
  return IDBF_OK;
}

namespace {
// device scratch for the gradient: (4 hidden + 2) n floats + the loss
struct MlpScratch {
  float* ws = nullptr;
  float* loss = nullptr;
  ~MlpScratch() {
    if (ws) (void)hipFree(ws);
    if (loss) (void)hipFree(loss);
  }
  idbf_status alloc(int hidden, int64_t n, int64_t nloss) {
    if (hipMalloc(&ws, size_t(4 * hidden + 2) * size_t(n) * sizeof(float)) != hipSuccess ||
        hipMalloc(&loss, size_t(nloss) * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("mlp: scratch allocation failed");
      return IDBF_ENOMEM;
    }
    return IDBF_OK;
  }
};
}  // namespace

idbf_status idbf_mlp_loss_grad(idbf_mlp m, const float* X, const float* y, int64_t n, float* grad, float* loss,
                               void* stream) {
  g_err[0] = 0;
  if (!m || n < 1 || !X || !y || !grad || !loss) {
    set_error("mlp_loss_grad: invalid arguments");
    return IDBF_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  MlpScratch sc;
  TRY(sc.alloc(m->hidden, n, 1));
  IDBF_HIP_CHECK(launch_mlp_loss_grad(m->P, kProposalInputs, m->hidden, X, y, n, grad, sc.loss, sc.ws, st));
  float sum = 0.f;
  IDBF_HIP_CHECK(hipMemcpyAsync(&sum, sc.loss, sizeof sum, hipMemcpyDeviceToHost, st));
  IDBF_HIP_CHECK(hipStreamSynchronize(st));
  *loss = 0.5f * sum / (float)n;
  return IDBF_OK;
}

idbf_status idbf_mlp_train(idbf_mlp m, const float* X, const float* y, int64_t n, int32_t epochs, int32_t batch,
                           float lr, uint64_t seed, float* loss_per_epoch, void* stream) {
  g_err[0] = 0;
  if (!m || n < 1 || n > INT32_MAX || !X || !y || epochs < 0 || batch < 1 || !(lr > 0.f)) {
    set_error("mlp_train: invalid arguments");
    return IDBF_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nb = (n + batch - 1) / batch;
  MlpScratch sc;
  TRY(sc.alloc(m->hidden, batch, nb));
  float *Xb = nullptr, *yb = nullptr, *G = nullptr;
  int32_t* idx = nullptr;
  struct Free {
    std::vector<void*> p;
    ~Free() {
      for (void* q : p) (void)hipFree(q);
    }
  } fr;
  auto dev = [&](void** p, size_t bytes) -> idbf_status {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("mlp_train: allocation failed");
      return IDBF_ENOMEM;
    }
    fr.p.push_back(*p);
    return IDBF_OK;
  };
  TRY(dev(reinterpret_cast<void**>(&Xb), size_t(batch) * kProposalInputs * sizeof(float)));
  TRY(dev(reinterpret_cast<void**>(&yb), size_t(batch) * sizeof(float)));
  TRY(dev(reinterpret_cast<void**>(&G), size_t(m->np) * sizeof(float)));
  TRY(dev(reinterpret_cast<void**>(&idx), size_t(n) * sizeof(int32_t)));
  std::vector<int32_t> perm(n);
  std::vector<float> losses(nb);
  for (int32_t e = 0; e < epochs; ++e) {
    // Fisher-Yates with SplitMix64 draws (counter: seed, epoch, position)
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
      uint64_t z = (seed ^ (uint64_t(e) << 40)) + uint64_t(i) + 0x9E3779B97F4A7C15ull;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      const int64_t j = (int64_t)(((z >> 32) * uint64_t(i + 1)) >> 32);
      std::swap(perm[i], perm[j]);
    }
    IDBF_HIP_CHECK(hipMemcpyAsync(idx, perm.data(), size_t(n) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    for (int64_t bi = 0; bi < nb; ++bi) {
      const int64_t b0 = bi * batch, rows = std::min<int64_t>(batch, n - b0);
      IDBF_HIP_CHECK(launch_gather_rows(X, y, idx + b0, rows, kProposalInputs, Xb, yb, st));
      IDBF_HIP_CHECK(launch_mlp_loss_grad(m->P, kProposalInputs, m->hidden, Xb, yb, rows, G, sc.loss + bi, sc.ws, st));
      IDBF_HIP_CHECK(launch_adam(m->P, G, m->M, m->V, m->np, lr, ++m->step, st));
    }
    IDBF_HIP_CHECK(hipMemcpyAsync(losses.data(), sc.loss, size_t(nb) * sizeof(float), hipMemcpyDeviceToHost, st));
    IDBF_HIP_CHECK(hipStreamSynchronize(st));  // also keeps perm alive until its copy is done
    double sum = 0.0;
    for (float v : losses) sum += v;
    if (loss_per_epoch) loss_per_epoch[e] = (float)(0.5 * sum / (double)n);
  }
  IDBF_HIP_CHECK(hipStreamSynchronize(st));
  return IDBF_OK;
}

idbf_status idbf_rank_samples(idbf_handle h, int32_t side, int32_t level, float* features, float* targets) {
  g_err[0] = 0;
  const Batch* b = h ? find_batch(h, side, level) : nullptr;
  if (!b || !features || !targets) {
    set_error("rank_samples: invalid handle, side, level or NULL output");
    return IDBF_EINVAL;
  }
  IDBF_HIP_CHECK(launch_features(b->n, h->L, level, side == IDBF_SIDE_U ? 0 : 1, h->ph, features, h->stream));
  IDBF_HIP_CHECK(launch_rank_targets(b->rank, b->n, targets, h->stream));
  IDBF_HIP_CHECK(hipStreamSynchronize(h->stream));
  return IDBF_OK;
}

}  // extern "C"

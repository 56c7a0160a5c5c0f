// C ABI of libpft: argument validation, temporary memory, launch sequencing.
//
// Every entry point validates its arguments synchronously, takes temporary
// device memory from the stream-ordered allocator on the caller's stream,
// enqueues the prologue / compute / finish kernels on that stream and returns.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "pft_internal.h"

using namespace pft;

namespace {

thread_local std::string g_err;

pft_status fail(pft_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

pft_status hip_fail(hipError_t e, const char* what) {
  return fail(PFT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

size_t real_size(int dt) { return dt == PFT_F64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// stream-ordered temporaries
// ---------------------------------------------------------------------------
std::mutex g_pool_mu;
std::vector<int> g_pool_ready;

void ensure_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (std::find(g_pool_ready.begin(), g_pool_ready.end(), dev) != g_pool_ready.end()) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;  // keep freed blocks cached across calls
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  g_pool_ready.push_back(dev);
}

// Temporary device memory of one call. Each (device, stream) pair keeps a
// workspace that calls on that stream reuse: stream order makes a call's kernels
// finish before the next call's kernels touch the same bytes, and the workspace
// mutex (held from construction to destruction, i.e. while the call enqueues its
// work) keeps two host threads from interleaving their work on one stream. A
// call that needs more than the workspace holds takes the rest from the
// stream-ordered allocator and grows the workspace for the next call, so in a
// steady loop no allocation or free is issued at all (freeing stream-ordered
// memory was measured to block the host for about 0.17 ms per free here). An
// Arena created while the same thread already holds the stream's workspace
// (a nested call) uses the stream-ordered allocator only.
struct Workspace {
  std::mutex mu;
  std::atomic<std::thread::id> owner{std::thread::id()};
  char* base = nullptr;
  size_t cap = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;

Workspace* workspace_for(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  std::unique_ptr<Workspace>& w = g_ws[{dev, s}];
  if (!w) w.reset(new Workspace);
  return w.get();
}

struct Arena {
  explicit Arena(hipStream_t s) : s_(s) {
    Workspace* w = workspace_for(s);
    if (w && w->owner.load() != std::this_thread::get_id()) {
      w->mu.lock();
      w->owner.store(std::this_thread::get_id());
      ws_ = w;
    }
  }
  // A fixed buffer of `cap` device bytes that the caller owns: get() carves from it and fails
  // (failed = true) past its end; nothing is ever allocated or freed.
  Arena(hipStream_t s, char* base, size_t cap) : s_(s), fixed_(base), fixed_cap_(cap) {}
  ~Arena() {
    if (fixed_) return;
    for (void* p : ptrs_) (void)hipFreeAsync(p, s_);
    if (!ws_) return;
    if (need_ > ws_->cap) {  // grow for the next call (the old block is freed after this call's work)
      if (ws_->base) (void)hipFreeAsync(ws_->base, s_);
      ws_->base = nullptr;
      ws_->cap = 0;
      const size_t cap = need_ + need_ / 4;
      void* b = nullptr;
      if (hipMallocAsync(&b, cap, s_) == hipSuccess && b != nullptr) {
        ws_->base = static_cast<char*>(b);
        ws_->cap = cap;
      }
    }
    ws_->owner.store(std::thread::id());
    ws_->mu.unlock();
  }
  // bytes that get<T>(count) takes
  template <typename T>
  static size_t take(size_t count) {
    return (std::max<size_t>(count * sizeof(T), 256) + 255) / 256 * 256;
  }
  template <typename T>
  T* get(size_t count) {
    const size_t bytes = take<T>(count);
    need_ += bytes;
    if (fixed_) {
      if (used_ + bytes > fixed_cap_) {
        failed = true;
        return nullptr;
      }
      T* p = reinterpret_cast<T*>(fixed_ + used_);
      used_ += bytes;
      return p;
    }
    if (ws_ && ws_->base && used_ + bytes <= ws_->cap) {
      T* p = reinterpret_cast<T*>(ws_->base + used_);
      used_ += bytes;
      return p;
    }
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, s_) != hipSuccess || p == nullptr) {
      failed = true;
      return nullptr;
    }
    ptrs_.push_back(p);
    return static_cast<T*>(p);
  }
  bool failed = false;

 private:
  hipStream_t s_;
  Workspace* ws_ = nullptr;
  char* fixed_ = nullptr;
  size_t fixed_cap_ = 0;
  size_t used_ = 0, need_ = 0;
  std::vector<void*> ptrs_;
};

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
struct ProfRec {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> done;
  hipEvent_t open = nullptr;
  int64_t launches = 0;
  double total_ms = 0.0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, ProfRec> g_prof;

// ---------------------------------------------------------------------------
// heuristics
// ---------------------------------------------------------------------------
#ifndef PFT_TARGET_BLOCKS
#define PFT_TARGET_BLOCKS 16384
#endif
constexpr int64_t kTargetBlocks = PFT_TARGET_BLOCKS;  // 64 blocks of 256 threads per CU on 256 CUs: short tails
#ifndef PFT_TARGET_BLOCKS_F32
#define PFT_TARGET_BLOCKS_F32 49152
#endif
// the same for the FP32C forward's face splits: its blocks of four wavefronts share one Q-tile and exit
// wavefront by wavefront, and three times as many (shorter) blocks measured 1.5-4 % faster on the larger
// workloads (2.1M Q x 1e5 faces, 65 536 Q x 81 920 faces); the adjoint keeps kTargetBlocks
constexpr int64_t kTargetBlocksF32 = PFT_TARGET_BLOCKS_F32;
#ifndef PFT_MIN_FACES_PER_SPLIT
#define PFT_MIN_FACES_PER_SPLIT 128
#endif
constexpr int64_t kMinFacesPerSplit = PFT_MIN_FACES_PER_SPLIT;
#ifndef PFT_BATCH_CHUNK_F
#define PFT_BATCH_CHUNK_F 512
#endif
#ifndef PFT_BATCH_CHUNK_Q
#define PFT_BATCH_CHUNK_Q 65536
#endif
constexpr int64_t kBatchChunkF = PFT_BATCH_CHUNK_F;  // faces per batched forward item
#ifndef PFT_BATCH_PARTIAL_CAP_MIB
#define PFT_BATCH_PARTIAL_CAP_MIB 4096
#endif
// Device memory the batched forward's partial slots (Q x face chunks, 16 B each) may take: with more, the
// face chunks are made longer (fewer slots) and tuner candidates beyond it are not tried.
constexpr int64_t kBatchPartialCapBytes = (int64_t)PFT_BATCH_PARTIAL_CAP_MIB << 20;
constexpr int64_t kBatchChunkQ = PFT_BATCH_CHUNK_Q;  // Q per batched adjoint item

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// tile sizes of the batched launches, tuned at run time
// ---------------------------------------------------------------------------
// The batched forward's Q per thread and faces per work item, and the batched
// adjoint's Q per work item, are chosen per (GPU, form, size bucket): the
// first call whose key is new runs every candidate once on its own input, times
// each with events (a synchronous call), keeps the fastest, and produces its
// output with it; later calls with that key use the kept choice. With
// PFT_AUTOTUNE=0 in the environment the compiled defaults are used.
struct BatchTiles {
  int qpt = kQPTBatch;
  int64_t chunk_f = kBatchChunkF;
  int64_t chunk_q = kBatchChunkQ;
};
std::mutex g_tune_mu;
std::map<std::string, BatchTiles> g_tuned;
std::vector<std::string> g_tune_log;
thread_local std::string g_tune_text;

bool autotune_enabled() {
  const char* e = std::getenv("PFT_AUTOTUNE");
  return e == nullptr || e[0] != '0';
}

int log2_bucket(double x) { return x > 1.0 ? (int)std::floor(std::log2(x)) : 0; }

std::string tune_key(const char* what, int mode, bool share, int64_t n_meshes, double pairs, int64_t nf) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  return std::string(what) + "[" + arch + (mode == PFT_FP64 ? ",fp64" : ",fp32c") + (share ? ",edge-sharing" : "") +
         ",meshes~2^" + std::to_string(log2_bucket((double)n_meshes)) + ",faces~2^" +
         std::to_string(log2_bucket((double)nf)) + ",pairs~2^" + std::to_string(log2_bucket(pairs)) + "]";
}

bool tuned_tiles(const std::string& key, BatchTiles* t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(key);
  if (it == g_tuned.end()) return false;
  *t = it->second;
  return true;
}

void keep_tiles(const std::string& key, const BatchTiles& t, const std::string& log) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = t;
  g_tune_log.push_back(log);
}

// Time each candidate (enqueued by run(candidate)) on stream s; returns the index of the fastest, or
// -1 if timing failed (the caller then uses its first candidate).
template <typename F>
int time_candidates(int n, F run, hipStream_t s, std::vector<float>& ms) {
  std::vector<hipEvent_t> ev(2 * n, nullptr);
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) e = nullptr;
  int best = -1;
  bool ok = true;
  for (int i = 0; i < n && ok; ++i) {
    ok = ev[2 * i] && ev[2 * i + 1] && hipEventRecord(ev[2 * i], s) == hipSuccess;
    ok = ok && run(i) == PFT_OK && hipEventRecord(ev[2 * i + 1], s) == hipSuccess;
  }
  ms.assign(n, 0.0f);
  if (ok && hipEventSynchronize(ev[2 * n - 1]) == hipSuccess) {
    for (int i = 0; i < n; ++i) {
      if (hipEventElapsedTime(&ms[i], ev[2 * i], ev[2 * i + 1]) != hipSuccess) ms[i] = 1e30f;
      if (best < 0 || ms[i] < ms[best]) best = i;
    }
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return best;
}

// Face splits of a Q-parallel forward whose blocks hold qtile Q each: about `target` blocks, with at
// least min_faces faces per split.
void choose_face_splits(int64_t nq, int64_t nf, int64_t qtile, int64_t min_faces, int64_t target, int* splits,
                        int64_t* per) {
  if (nf <= 0) {
    *splits = 1;
    *per = 0;
    return;
  }
  const int64_t qblocks = cdiv(nq, qtile);
  int64_t s = std::max<int64_t>(1, std::min(cdiv(target, qblocks), cdiv(nf, min_faces)));
  int64_t p = cdiv(cdiv(nf, s), kTileF) * kTileF;
  *per = p;
  *splits = (int)cdiv(nf, p);
}

// Face splits of a single-mesh forward (sets a.splits and a.faces_per_split; returns the double2 partial
// entries they need), capped so that the partials fit in max_partials entries when that is > 0.
int64_t plan_forward(int64_t nq, int64_t nf, bool c128, int64_t max_partials, FwdArgs& a) {
  int splits;
  int64_t per;
  a.qpt = fwd_qpt(nq);
  choose_face_splits(nq, nf, c128 ? kBlock : fwd_qtile(a.qpt),
                     c128 ? kMinFacesPerSplit : kMinFacesPerSplit * kFwdSplitWaves,
                     c128 ? kTargetBlocks : kTargetBlocksF32, &splits, &per);
  if (max_partials > 0 && (int64_t)splits * nq > max_partials && nf > 0) {
    const int64_t cap = std::max<int64_t>(1, max_partials / nq);
    per = cdiv(cdiv(nf, cap), kTileF) * kTileF;
    splits = (int)cdiv(nf, per);
  }
  a.splits = splits;
  a.faces_per_split = per;
  return (int64_t)splits * nq;
}

// Q-splits of the vertex adjoint (blocks of `tile` faces): about kTargetBlocks blocks, at least kBlock Q per
// split; from kXcds splits up, a multiple of kXcds, so that each die takes whole Q-splits.
void choose_q_splits(int64_t nq, int64_t nf, int tile, int* splits, int64_t* per) {
  const int64_t fblocks = std::max<int64_t>(1, cdiv(nf, tile));
  const int64_t smax = std::max<int64_t>(1, cdiv(nq, kBlock));
  int64_t s = std::max<int64_t>(1, std::min(cdiv(kTargetBlocks, fblocks), smax));
  if (s >= kXcds) {
    s = cdiv(s, kXcds) * kXcds;
    if (s > smax) s -= kXcds;
  }
  const int64_t p = std::max<int64_t>(1, cdiv(nq, s));
  *per = p;
  *splits = (int)std::max<int64_t>(1, cdiv(nq, p));
}

int num_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
// With PFT_VALIDATE=1 in the environment, the single-mesh triangle entry points
// first check the mesh on the host (a synchronous copy of the triangles and
// vertices): indices in range, no repeated vertex, closed (every edge used by
// exactly two faces) and consistently oriented (the two faces of an edge run it
// in opposite directions), and a non-negative enclosed volume (outward); each
// region is checked on its own. They return EINVAL if the mesh fails.
bool strict_validation() {
  const char* e = std::getenv("PFT_VALIDATE");
  return e != nullptr && e[0] == '1';
}

// Edge counts of faces [f0, f1) of a host triangle list (the checks of pft_check_mesh).
void count_mesh(const int32_t* tris, int64_t f0, int64_t f1, int64_t nv, pft_mesh_check* c) {
  *c = pft_mesh_check{0, 0, 0, 0, 0};
  std::vector<std::pair<uint64_t, int>> he;  // (unordered vertex pair, direction)
  he.reserve((size_t)(f1 - f0) * 3);
  for (int64_t f = f0; f < f1; ++f) {
    const int32_t v[3] = {tris[3 * f], tris[3 * f + 1], tris[3 * f + 2]};
    bool ok = true;
    for (int k = 0; k < 3; ++k)
      if (v[k] < 0 || v[k] >= nv) {
        ++c->bad_index;
        ok = false;
      }
    if (!ok) continue;
    if (v[0] == v[1] || v[1] == v[2] || v[2] == v[0]) {
      ++c->repeated_vertex;
      continue;
    }
    for (int k = 0; k < 3; ++k) {
      const uint64_t a = (uint32_t)v[k], b = (uint32_t)v[(k + 1) % 3];
      he.emplace_back(a < b ? (a << 32) | b : (b << 32) | a, a < b ? 1 : -1);
    }
  }
  std::sort(he.begin(), he.end());
  for (size_t i = 0; i < he.size();) {
    size_t j = i;
    int dir = 0;
    while (j < he.size() && he[j].first == he[i].first) dir += he[j++].second;
    const size_t n = j - i;
    if (n == 1) ++c->open_edges;
    else if (n > 2) ++c->nonmanifold_edges;
    else if (dir != 0) ++c->misoriented_edges;
    i = j;
  }
}

// Signed volume of faces [f0, f1) (host arrays, coordinates relative to the vertex mean).
double signed_volume(const std::vector<double>& v, const int32_t* tris, int64_t f0, int64_t f1) {
  const int64_t nv = (int64_t)v.size() / 3;
  double t[3] = {0.0, 0.0, 0.0};
  for (int64_t i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) t[k] += v[3 * i + k] / (double)nv;
  double vol = 0.0;
  for (int64_t f = f0; f < f1; ++f) {
    double p[3][3];
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) p[j][k] = v[3 * (int64_t)tris[3 * f + j] + k] - t[k];
    vol += (p[0][0] * (p[1][1] * p[2][2] - p[1][2] * p[2][1]) - p[0][1] * (p[1][0] * p[2][2] - p[1][2] * p[2][0]) +
            p[0][2] * (p[1][0] * p[2][1] - p[1][1] * p[2][0])) / 6.0;
  }
  return vol;
}

// The PFT_VALIDATE=1 check of a device mesh; region_offsets NULL: one region of all faces.
pft_status strict_mesh(const void* verts, int vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                       const int64_t* region_offsets, int64_t nreg, void* stream) {
  if (!strict_validation() || nf == 0) return PFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(s);
  std::vector<int32_t> t((size_t)nf * 3);
  std::vector<double> v((size_t)nv * 3);
  if (e == hipSuccess) e = hipMemcpy(t.data(), tris, t.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess && nv > 0) {
    if (vdtype == PFT_F64) {
      e = hipMemcpy(v.data(), verts, v.size() * sizeof(double), hipMemcpyDeviceToHost);
    } else {
      std::vector<float> vf(v.size());
      e = hipMemcpy(vf.data(), verts, vf.size() * sizeof(float), hipMemcpyDeviceToHost);
      for (size_t i = 0; i < vf.size(); ++i) v[i] = vf[i];
    }
  }
  if (e != hipSuccess) return hip_fail(e, "mesh check copy (PFT_VALIDATE=1)");
  const int64_t nr = region_offsets ? nreg : 1;
  for (int64_t r = 0; r < nr; ++r) {
    const int64_t f0 = region_offsets ? region_offsets[r] : 0, f1 = region_offsets ? region_offsets[r + 1] : nf;
    if (f1 <= f0) continue;
    pft_mesh_check c;
    count_mesh(t.data(), f0, f1, nv, &c);
    const std::string where = region_offsets ? " in region " + std::to_string(r) : std::string();
    if (c.bad_index || c.repeated_vertex || c.open_edges || c.nonmanifold_edges || c.misoriented_edges)
      return fail(PFT_EINVAL, "mesh not closed and consistently oriented" + where + " (PFT_VALIDATE=1): " +
                                  std::to_string(c.bad_index) + " indices out of range, " +
                                  std::to_string(c.repeated_vertex) + " faces with a repeated vertex, " +
                                  std::to_string(c.open_edges) + " open edges, " +
                                  std::to_string(c.nonmanifold_edges) + " edges of more than two faces, " +
                                  std::to_string(c.misoriented_edges) + " edges run the same way by both faces");
    if (signed_volume(v, t.data(), f0, f1) < 0.0)
      return fail(PFT_EINVAL, "mesh oriented inward (negative enclosed volume)" + where + " (PFT_VALIDATE=1)");
  }
  return PFT_OK;
}

pft_status check_mesh_args(const void* verts, int vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                           const void* q, int qdtype, int64_t nq, int mode) {
  if (mode != PFT_FP64 && mode != PFT_FP32C) return fail(PFT_EUNSUPPORTED, "unknown mode");
  if (vdtype != PFT_F32 && vdtype != PFT_F64) return fail(PFT_EUNSUPPORTED, "unknown vertex dtype");
  if (qdtype != PFT_F32 && qdtype != PFT_F64) return fail(PFT_EUNSUPPORTED, "unknown q dtype");
  if (nv < 0 || nf < 0 || nq < 0) return fail(PFT_EINVAL, "negative count");
  if (nv > INT32_MAX || nf > INT32_MAX / 3) return fail(PFT_EINVAL, "mesh too large for 32-bit indices");
  if (nv > 0 && verts == nullptr) return fail(PFT_EINVAL, "verts is NULL");
  if (nf > 0 && tris == nullptr) return fail(PFT_EINVAL, "tris is NULL");
  if (nq > 0 && q == nullptr) return fail(PFT_EINVAL, "q is NULL");
  if (verts && !aligned(verts, real_size(vdtype))) return fail(PFT_EINVAL, "verts misaligned");
  if (tris && !aligned(tris, 4)) return fail(PFT_EINVAL, "tris misaligned");
  if (q && !aligned(q, real_size(qdtype))) return fail(PFT_EINVAL, "q misaligned");
  return PFT_OK;
}

pft_status check_offsets(const int64_t* off, int64_t n, const char* name) {
  if (off == nullptr) return fail(PFT_EINVAL, std::string(name) + " is NULL");
  if (off[0] != 0) return fail(PFT_EINVAL, std::string(name) + "[0] must be 0");
  for (int64_t i = 0; i < n; ++i)
    if (off[i + 1] < off[i]) return fail(PFT_EINVAL, std::string(name) + " must be non-decreasing");
  return PFT_OK;
}

hipError_t zero_bytes(void* p, size_t bytes, hipStream_t s) {
  // all outputs are multiples of 4 bytes
  return launch_zero_u32(static_cast<uint32_t*>(p), (int64_t)(bytes / 4), s);
}

const char* main_name(bool fwd, int mode) {
  if (fwd) return mode == PFT_FP64 ? "fwd3d_fp64" : "fwd3d_fp32c";
  return mode == PFT_FP64 ? "bwd3d_fp64" : "bwd3d_fp32c";
}

template <typename T>
pft_status upload(Arena& ar, const std::vector<T>& v, T** d, hipStream_t s) {
  *d = ar.get<T>(std::max<size_t>(v.size(), 1));
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  if (v.empty()) return PFT_OK;
  hipError_t e = hipMemcpyAsync(*d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s);
  return e == hipSuccess ? PFT_OK : hip_fail(e, "upload");
}

// Visiting order of Q (qorder.hip): nearby Q share wavefronts. Below kQOrderMin Q
// the caller's order is kept (the sort would cost more than it saves).
#ifndef PFT_QORDER_MIN
#define PFT_QORDER_MIN 8192
#endif
constexpr int64_t kQOrderMin = PFT_QORDER_MIN;

pft_status build_qorder(Arena& ar, const void* q, int qdtype, int64_t nq, const int64_t* d_q_off, int64_t n_meshes,
                        uint32_t** perm, hipStream_t s) {
  *perm = nullptr;
  if (nq < kQOrderMin || nq > INT32_MAX) return PFT_OK;
  QOrderScratch w;
  w.box_partial = ar.get<double>(256 * 6);
  w.box = ar.get<double>(6);
  w.keys = ar.get<uint64_t>(nq);
  w.keys_sorted = ar.get<uint64_t>(nq);
  w.vals = ar.get<uint32_t>(nq);
  w.perm = ar.get<uint32_t>(nq);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  hipError_t e = qorder_sort_bytes(nq, n_meshes, &w.sort_bytes);
  if (e != hipSuccess) return hip_fail(e, "Q sort size query");
  w.sort_temp = ar.get<unsigned char>(w.sort_bytes);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  e = launch_qorder(q, qdtype, nq, d_q_off, n_meshes, w, s);
  if (e != hipSuccess) return hip_fail(e, "Q order");
  *perm = w.perm;
  return PFT_OK;
}

// The adjoint's Q records: Q in visiting order with their centred cotangents
// (binary32 records for FP32C, binary64 records for FP64; the other is NULL).
// A caller's Q visiting order (a permutation of 0 .. nq-1), clamped into range on the device.
pft_status caller_qorder(Arena& ar, const uint32_t* q_order, int64_t nq, uint32_t** perm, hipStream_t s) {
  *perm = ar.get<uint32_t>(std::max<int64_t>(nq, 1));
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  hipError_t e = launch_clamp_perm(q_order, nq, *perm, s);
  return e == hipSuccess ? PFT_OK : hip_fail(e, "Q order");
}

// The same records for a visiting order already built (perm NULL: the caller's order).
pft_status qrecs_from_perm(Arena& ar, int mode, const void* q, int qdtype, const void* grad_out, int64_t nq,
                           const MeshInfo* info, const int64_t* d_q_off, int64_t n_meshes, uint32_t* perm,
                           QRec32** rec, QRec64** rec64, hipStream_t s) {
  *rec = nullptr;
  *rec64 = nullptr;
  if (!perm) {  // identity order
    perm = ar.get<uint32_t>(nq);
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    hipError_t e = launch_iota_u32(perm, nq, s);
    if (e != hipSuccess) return hip_fail(e, "Q order");
  }
  hipError_t e;
  if (mode == PFT_FP64) {
    *rec64 = ar.get<QRec64>(nq);
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    e = launch_qrec64_gather(q, qdtype, grad_out, nq, perm, info, d_q_off, n_meshes, *rec64, s);
  } else {
    *rec = ar.get<QRec32>(nq);
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    e = launch_qrec32_gather(q, qdtype, grad_out, nq, perm, info, d_q_off, n_meshes, *rec, s);
  }
  return e == hipSuccess ? PFT_OK : hip_fail(e, "Q records");
}

pft_status build_qrecs(Arena& ar, int mode, const void* q, int qdtype, const void* grad_out, int64_t nq,
                       const MeshInfo* info, const int64_t* d_q_off, int64_t n_meshes, QRec32** rec,
                       QRec64** rec64, hipStream_t s) {
  uint32_t* perm = nullptr;
  pft_status st = build_qorder(ar, q, qdtype, nq, d_q_off, n_meshes, &perm, s);
  if (st != PFT_OK) return st;
  return qrecs_from_perm(ar, mode, q, qdtype, grad_out, nq, info, d_q_off, n_meshes, perm, rec, rec64, s);
}

// Shared tail of the adjoint: per-corner vectors -> sorted incidence -> vertex gather.
pft_status gather_tail(Arena& ar, const int32_t* tris, int64_t nf, const int64_t* d_vert_off,
                       const int32_t* d_face_mesh, int64_t nv_total, const double* contrib, void* grad, int vdtype,
                       hipStream_t s) {
  const int64_t ns = nf * 3;
  uint32_t* keys = ar.get<uint32_t>(ns);
  uint32_t* vals = ar.get<uint32_t>(ns);
  uint32_t* keys_s = ar.get<uint32_t>(ns);
  uint32_t* vals_s = ar.get<uint32_t>(ns);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  hipError_t e = launch_incidence_keys(tris, nf, d_vert_off, d_face_mesh, nv_total, keys, vals, s);
  if (e != hipSuccess) return hip_fail(e, "incidence keys");
  size_t tb = 0;
  e = sort_incidence(keys, vals, keys_s, vals_s, ns, nv_total, nullptr, &tb, s);
  if (e != hipSuccess) return hip_fail(e, "sort size query");
  void* temp = ar.get<unsigned char>(tb);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  e = sort_incidence(keys, vals, keys_s, vals_s, ns, nv_total, temp, &tb, s);
  if (e != hipSuccess) return hip_fail(e, "incidence sort");
  e = launch_gather_vertices(keys_s, vals_s, ns, contrib, nv_total, grad, vdtype, s);
  if (e != hipSuccess) return hip_fail(e, "vertex gather");
  return PFT_OK;
}

}  // namespace

namespace pft {

void prof_begin(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  ProfRec& r = g_prof[name];
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  r.open = e;
}

void prof_end(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  ProfRec& r = g_prof[name];
  if (!r.open) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  r.done.emplace_back(r.open, e);
  r.open = nullptr;
}

}  // namespace pft

extern "C" {

const char* pft_version(void) { return "pft 0.1.0 (gfx950)"; }

const char* pft_last_error(void) { return g_err.c_str(); }

pft_status pft_release_workspace(void) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipMemPool_t pool;
  e = hipDeviceGetDefaultMemPool(&pool, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetDefaultMemPool");
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  {  // the per-stream workspaces of this device (none is in use: the calls that hold them are synchronous)
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto& kv : g_ws) {
      if (kv.first.first != dev || !kv.second) continue;
      std::lock_guard<std::mutex> wl(kv.second->mu);
      if (kv.second->base) (void)hipFree(kv.second->base);
      kv.second->base = nullptr;
      kv.second->cap = 0;
    }
  }
  e = hipMemPoolTrimTo(pool, 0);
  if (e != hipSuccess) return hip_fail(e, "hipMemPoolTrimTo");
  return PFT_OK;
}

const char* pft_tuning_info(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_text.clear();
  for (const std::string& l : g_tune_log) g_tune_text += l + "\n";
  return g_tune_text.c_str();
}

pft_status pft_profile_enable(int enable) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = enable != 0;
  return PFT_OK;
}

pft_status pft_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& kv : g_prof) {
    for (auto& pr : kv.second.done) {
      (void)hipEventSynchronize(pr.second);
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    if (kv.second.open) (void)hipEventDestroy(kv.second.open);
  }
  g_prof.clear();
  return PFT_OK;
}

pft_status pft_profile_read(const char* name, int64_t* launches, double* total_ms) {
  if (!name) return fail(PFT_EINVAL, "name is NULL");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  auto it = g_prof.find(name);
  int64_t n = 0;
  double ms = 0.0;
  if (it != g_prof.end()) {
    ProfRec& r = it->second;
    for (auto& pr : r.done) {
      hipError_t e = hipEventSynchronize(pr.second);
      if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
      float t = 0.0f;
      e = hipEventElapsedTime(&t, pr.first, pr.second);
      if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      r.total_ms += t;
      r.launches += 1;
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    r.done.clear();
    n = r.launches;
    ms = r.total_ms;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  return PFT_OK;
}

pft_status pft_validate_mesh(const int32_t* tris, int64_t nf, int64_t nv, int64_t* n_bad_index,
                             int64_t* n_repeated_vertex, void* stream) {
  if (nf < 0 || nv < 0) return fail(PFT_EINVAL, "negative count");
  if (nf > 0 && tris == nullptr) return fail(PFT_EINVAL, "tris is NULL");
  if (tris && !aligned(tris, 4)) return fail(PFT_EINVAL, "tris misaligned");
  int64_t bad = 0, rep = 0;
  if (nf > 0) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    ensure_pool();
    unsigned long long host[2] = {0, 0};
    {
      Arena ar(s);
      unsigned long long* d = ar.get<unsigned long long>(2);
      if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
      hipError_t e = launch_zero_u32(reinterpret_cast<uint32_t*>(d), 4, s);
      if (e == hipSuccess) e = launch_validate(tris, nf, nv, d, s);
      if (e == hipSuccess) e = hipMemcpyAsync(host, d, sizeof(host), hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return hip_fail(e, "validate");
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    bad = (int64_t)host[0];
    rep = (int64_t)host[1];
  }
  if (n_bad_index) *n_bad_index = bad;
  if (n_repeated_vertex) *n_repeated_vertex = rep;
  return PFT_OK;
}

pft_status pft_forward_2d(const double* verts, int64_t nv, const int64_t* contour_offsets, int64_t ncontours,
                          const double* q, int64_t nq, double* out, void* stream) {
  if (nv < 0 || nq < 0) return fail(PFT_EINVAL, "negative count");
  if (nv > 0 && verts == nullptr) return fail(PFT_EINVAL, "verts is NULL");
  if (nq > 0 && (q == nullptr || out == nullptr)) return fail(PFT_EINVAL, "q or out is NULL");
  if ((verts && !aligned(verts, 8)) || (q && !aligned(q, 8)) || (out && !aligned(out, 8)))
    return fail(PFT_EINVAL, "pointer misaligned (8 bytes required)");
  if (contour_offsets) {
    if (ncontours < 0) return fail(PFT_EINVAL, "negative contour count");
    pft_status st = check_offsets(contour_offsets, ncontours, "contour_offsets");
    if (st != PFT_OK) return st;
    if (contour_offsets[ncontours] != nv) return fail(PFT_EINVAL, "contour_offsets must end at nv");
  }
  if (nq == 0) return PFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  Arena ar(s);
  MeshInfo* info = ar.get<MeshInfo>(1);
  Edge2D* edges = ar.get<Edge2D>(std::max<int64_t>(nv, 1));
  int64_t* d_off = nullptr;
  if (contour_offsets) d_off = ar.get<int64_t>(ncontours + 1);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  hipError_t e = hipSuccess;
  if (d_off)
    e = hipMemcpyAsync(d_off, contour_offsets, sizeof(int64_t) * (ncontours + 1), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "offsets upload");
  e = launch_edges2d(verts, nv, d_off, ncontours, info, edges, s);
  if (e != hipSuccess) return hip_fail(e, "2D prologue");
  prof_begin("fwd2d_fp64", s);
  e = launch_fwd2d(edges, nv, info, 0.0, q, nq, kTau02D, out, s);
  prof_end("fwd2d_fp64", s);
  if (e != hipSuccess) return hip_fail(e, "2D transform");
  return PFT_OK;
}

}  // extern "C"

namespace {

// The 3D forward after validation: prologue, Q order, transform, finish.
// `out` may be NULL when only |F|^2 is wanted.
// sort_q = false with no q_order visits Q in the list order (no sort temporaries); max_partials > 0 caps
// splits * nq (a fixed scratch); profile = false records no timing events.
pft_status forward3d_core(Arena& ar, const void* verts, int vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                          const void* q, int qdtype, int64_t nq, int mode, void* out, void* intensity,
                          hipStream_t s, const int32_t* order = nullptr, const uint8_t* meta = nullptr,
                          const uint32_t* q_order = nullptr, bool sort_q = true, int64_t max_partials = -1,
                          bool profile = true) {
  const bool c128 = mode == PFT_FP64;
  pft_status st = PFT_OK;
  MeshInfo* info = ar.get<MeshInfo>(1);
  Face64* f64 = ar.get<Face64>(std::max<int64_t>(nf, 1));
  Face32* f32 = c128 ? nullptr : ar.get<Face32>(std::max<int64_t>(nf, 1));
  FwdArgs a;
  const int64_t n_partial = plan_forward(nq, nf, c128, max_partials, a);
  double2* partial = ar.get<double2>((size_t)n_partial);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  hipError_t e = launch_mesh_info_single(verts, vdtype, 3, nv, info, s);
  if (e == hipSuccess)
    e = launch_face64(verts, vdtype, nv, tris, nf, info, c128 ? kTauF64 : kTauF32, f64, s, order, meta);
  if (e == hipSuccess && !c128) e = launch_face32(f64, nf, kTauF32, kTauRel32, f32, s);
  if (e != hipSuccess) return hip_fail(e, "3D prologue");
  uint32_t* perm = nullptr;
  if (q_order)
    st = caller_qorder(ar, q_order, nq, &perm, s);
  else if (sort_q)
    st = build_qorder(ar, q, qdtype, nq, nullptr, 1, &perm, s);
  if (st != PFT_OK) return st;
  a.f64 = f64;
  a.f32 = f32;
  a.info = info;
  a.nf = nf;
  a.q = q;
  a.qdtype = qdtype;
  a.nq = nq;
  a.perm = perm;
  a.split_face = nullptr;
  a.partial = partial;
  a.out = out;
  a.intensity = intensity;
  a.tau0 = c128 ? kTau0F64 : kTau0F32;
  a.share_edges = (order != nullptr && !c128) ? 1 : 0;
  const char* nm = main_name(true, mode);
  if (profile) prof_begin(nm, s);
  e = c128 ? launch_fwd3d_fp64(a, s) : launch_fwd3d_fp32c(a, s);
  if (profile) prof_end(nm, s);
  if (e != hipSuccess) return hip_fail(e, "3D transform");
  e = launch_fwd3d_finish(a, c128 ? 1 : 0, s);
  if (e != hipSuccess) return hip_fail(e, "3D finish");
  return PFT_OK;
}

// ---------------------------------------------------------------------------
// closed regions of constant density
// ---------------------------------------------------------------------------
constexpr int64_t kMaxRegions = 4096;

pft_status check_regions(const int64_t* off, int64_t nreg, int64_t nf, const double* rho) {
  if (nreg < 0 || nreg > kMaxRegions) return fail(PFT_EINVAL, "nreg must be 0 .. 4096");
  pft_status st = check_offsets(off, nreg, "region_offsets");
  if (st != PFT_OK) return st;
  if (off[nreg] != nf) return fail(PFT_EINVAL, "region_offsets must end at nf");
  if (nreg > 0 && rho == nullptr) return fail(PFT_EINVAL, "rho is NULL");
  if (rho && !aligned(rho, 8)) return fail(PFT_EINVAL, "rho misaligned");
  return PFT_OK;
}

// Face splits that never cross a region boundary: each non-empty region gets
// about nf_j / per splits (per as for one mesh), so every split's partial sum
// belongs to one region and the finish kernels can weight and separate them.
struct RegionPlan {
  std::vector<int64_t> split_face;   // [splits + 1]
  std::vector<int32_t> region_split; // [nreg + 1]
  int splits = 0;
  int64_t* d_split_face = nullptr;
  int32_t* d_region_split = nullptr;
};

// Each region's own radius about its centre (region_R) and, per split, its region's centre and radius
// (split_geo): the small-|Q| tests and the tetrahedron fan's apex use them, so that a region much smaller than the whole set is not summed by its
// surface form where that form cancels (|Q| times the region's size small).
pft_status region_radii(Arena& ar, const int64_t* off, int64_t nreg, const Face64* f64, const int32_t* d_region_split,
                        int splits, double** region_R, double4** split_geo, hipStream_t s) {
  *region_R = ar.get<double>(std::max<int64_t>(nreg, 1));
  double4* region_geo = ar.get<double4>(std::max<int64_t>(nreg, 1));
  *split_geo = ar.get<double4>(std::max(splits, 1));
  int64_t* d_off = nullptr;
  std::vector<int64_t> offv(off, off + nreg + 1);
  pft_status st = upload(ar, offv, &d_off, s);
  if (st != PFT_OK) return st;
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  hipError_t e = launch_region_radii(f64, d_off, (int)nreg, d_region_split, *region_R, region_geo, *split_geo, s);
  return e == hipSuccess ? PFT_OK : hip_fail(e, "region radii");
}

pft_status plan_regions(Arena& ar, const int64_t* off, int64_t nreg, int64_t nq, int64_t qtile, int64_t min_faces,
                        int64_t target, RegionPlan& p,
                        hipStream_t s) {
  const int64_t nf = off[nreg];
  int s0 = 0;
  int64_t per = 0;
  choose_face_splits(nq, nf, qtile, min_faces, target, &s0, &per);
  if (per <= 0) per = kTileF;
  for (int64_t j = 0; j < nreg; ++j) {
    p.region_split.push_back((int32_t)p.split_face.size());
    const int64_t n = off[j + 1] - off[j];
    if (n <= 0) continue;
    const int64_t pj = cdiv(cdiv(n, cdiv(n, per)), (int64_t)kTileF) * kTileF;
    for (int64_t f = off[j]; f < off[j + 1]; f += pj) p.split_face.push_back(f);
  }
  p.region_split.push_back((int32_t)p.split_face.size());
  p.splits = (int)p.split_face.size();
  p.split_face.push_back(nf);
  pft_status st = upload(ar, p.split_face, &p.d_split_face, s);
  if (st == PFT_OK) st = upload(ar, p.region_split, &p.d_region_split, s);
  return st;
}

}  // namespace

extern "C" {

pft_status pft_forward_3d(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                          const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, void* out, void* intensity,
                          void* stream) {
  pft_status st = check_mesh_args(verts, vdtype, nv, tris, nf, q, qdtype, nq, mode);
  if (st != PFT_OK) return st;
  const bool c128 = mode == PFT_FP64;
  if (nq > 0 && out == nullptr) return fail(PFT_EINVAL, "out is NULL");
  if (out && !aligned(out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "out misaligned");
  if (intensity && !aligned(intensity, c128 ? 8 : 4)) return fail(PFT_EINVAL, "intensity misaligned");
  if (nq == 0) return PFT_OK;
  if ((st = strict_mesh(verts, vdtype, nv, tris, nf, nullptr, 0, stream)) != PFT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  Arena ar(s);
  return forward3d_core(ar, verts, vdtype, nv, tris, nf, q, qdtype, nq, mode, out, intensity, s);
}

pft_status pft_forward_3d_ordered(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                  const int32_t* face_order, const uint8_t* face_meta, const void* q,
                                  pft_dtype qdtype, int64_t nq, pft_mode mode, void* out, void* intensity,
                                  const uint32_t* q_order, void* stream) {
  pft_status st = check_mesh_args(verts, vdtype, nv, tris, nf, q, qdtype, nq, mode);
  if (st != PFT_OK) return st;
  const bool c128 = mode == PFT_FP64;
  if ((face_order == nullptr) != (face_meta == nullptr)) return fail(PFT_EINVAL, "face_order and face_meta go together");
  if (face_order && !aligned(face_order, 4)) return fail(PFT_EINVAL, "face_order misaligned");
  if (q_order && !aligned(q_order, 4)) return fail(PFT_EINVAL, "q_order misaligned");
  if (nq > 0 && out == nullptr) return fail(PFT_EINVAL, "out is NULL");
  if (out && !aligned(out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "out misaligned");
  if (intensity && !aligned(intensity, c128 ? 8 : 4)) return fail(PFT_EINVAL, "intensity misaligned");
  if (nq == 0) return PFT_OK;
  if ((st = strict_mesh(verts, vdtype, nv, tris, nf, nullptr, 0, stream)) != PFT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  Arena ar(s);
  return forward3d_core(ar, verts, vdtype, nv, tris, nf, q, qdtype, nq, mode, out, intensity, s,
                        nf > 0 ? face_order : nullptr, nf > 0 ? face_meta : nullptr, q_order);
}

}  // extern "C"

namespace pft {

pft_status set_error(pft_status st, const char* msg) { return fail(st, msg); }

// pft_forward_3d with every temporary carved from `scratch` (cap bytes of device memory the caller
// keeps): the Q are visited in the list order (no sort), the face splits are capped so that the
// partial sums fit, and the PFT_VALIDATE check (synchronous) and timing events are not used.
// `scratch_fn` supplies the buffer once the arguments have been checked.
pft_status forward3d_noalloc(pft_status (*scratch_fn)(void**), size_t cap, const void* verts, int vdtype,
                             int64_t nv, const int32_t* tris, int64_t nf, const void* q, int qdtype, int64_t nq,
                             int mode, void* out, void* intensity, void* stream) {
  pft_status st = check_mesh_args(verts, vdtype, nv, tris, nf, q, qdtype, nq, mode);
  if (st != PFT_OK) return st;
  const bool c128 = mode == PFT_FP64;
  if (nq > 0 && out == nullptr) return fail(PFT_EINVAL, "out is NULL");
  if (out && !aligned(out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "out misaligned");
  if (intensity && !aligned(intensity, c128 ? 8 : 4)) return fail(PFT_EINVAL, "intensity misaligned");
  if (nq == 0) return PFT_OK;
  const size_t fixed = Arena::take<MeshInfo>(1) + Arena::take<Face64>(std::max<int64_t>(nf, 1)) +
                       (c128 ? 0 : Arena::take<Face32>(std::max<int64_t>(nf, 1)));
  const size_t per_face = sizeof(Face64) + (c128 ? 0 : sizeof(Face32));
  if (fixed + Arena::take<double2>((size_t)nq) > cap) {
    if (fixed + Arena::take<double2>(1) > cap)
      return fail(PFT_EINVAL, "mesh too large for the no-allocation scratch: " + std::to_string(nf) +
                                  " faces need " + std::to_string(fixed) + " of its " + std::to_string(cap) +
                                  " bytes (" + std::to_string(per_face) + " bytes per face)");
    return fail(PFT_EINVAL, "too many Q for the no-allocation scratch with this mesh: at most " +
                                std::to_string((cap - fixed) / sizeof(double2) - 16) + " Q (16 bytes per Q " +
                                "beside the face records)");
  }
  void* base = nullptr;
  if ((st = scratch_fn(&base)) != PFT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Arena ar(s, static_cast<char*>(base), cap);
  const int64_t max_partials = (int64_t)((cap - fixed) / sizeof(double2)) - 16;
  st = forward3d_core(ar, verts, vdtype, nv, tris, nf, q, qdtype, nq, mode, out, intensity, s, nullptr, nullptr,
                      nullptr, false, max_partials, false);
  if (st == PFT_OK && ar.failed) return fail(PFT_EINVAL, "no-allocation scratch exhausted");
  return st;
}

}  // namespace pft

extern "C" {

pft_status pft_q_order(const void* q, pft_dtype qdtype, int64_t nq, uint32_t* order, void* stream) {
  if (qdtype != PFT_F32 && qdtype != PFT_F64) return fail(PFT_EUNSUPPORTED, "unknown q dtype");
  if (nq < 0) return fail(PFT_EINVAL, "negative count");
  if (nq > UINT32_MAX) return fail(PFT_EINVAL, "too many Q for 32-bit order entries");
  if (nq > 0 && (q == nullptr || order == nullptr)) return fail(PFT_EINVAL, "q or order is NULL");
  if ((q && !aligned(q, real_size(qdtype))) || (order && !aligned(order, 4))) return fail(PFT_EINVAL, "argument misaligned");
  if (nq == 0) return PFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  Arena ar(s);
  uint32_t* perm = nullptr;
  pft_status st = build_qorder(ar, q, qdtype, nq, nullptr, 1, &perm, s);
  if (st != PFT_OK) return st;
  hipError_t e = perm ? hipMemcpyAsync(order, perm, sizeof(uint32_t) * nq, hipMemcpyDeviceToDevice, s)
                      : launch_iota_u32(order, nq, s);  // below the sorting size: the list order
  return e == hipSuccess ? PFT_OK : hip_fail(e, "Q order");
}

pft_status pft_check_mesh(const int32_t* tris, int64_t nf, int64_t nv, pft_mesh_check* report) {
  if (nf < 0 || nv < 0) return fail(PFT_EINVAL, "negative count");
  if (nf > INT32_MAX / 3 || nv > INT32_MAX) return fail(PFT_EINVAL, "mesh too large for 32-bit indices");
  if (report == nullptr || (nf > 0 && tris == nullptr)) return fail(PFT_EINVAL, "tris or report is NULL");
  count_mesh(tris, 0, nf, nv, report);
  return PFT_OK;
}

pft_status pft_fp32c_q_limit(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                             double* q_limit) {
  if (vdtype != PFT_F32 && vdtype != PFT_F64) return fail(PFT_EUNSUPPORTED, "unknown vertex dtype");
  if (nf < 0 || nv < 0) return fail(PFT_EINVAL, "negative count");
  if (q_limit == nullptr || (nf > 0 && tris == nullptr) || (nv > 0 && verts == nullptr))
    return fail(PFT_EINVAL, "verts, tris or q_limit is NULL");
  auto vert = [&](int32_t i, int k) {
    return vdtype == PFT_F64 ? static_cast<const double*>(verts)[3 * (int64_t)i + k]
                             : (double)static_cast<const float*>(verts)[3 * (int64_t)i + k];
  };
  // rho: the largest distance from a face's centroid to one of its vertices (faces with an index
  // outside [0, nv) are empty in the transform and skipped here)
  double rho2 = 0.0;
  for (int64_t f = 0; f < nf; ++f) {
    const int32_t* ix = tris + 3 * f;
    if (ix[0] < 0 || ix[1] < 0 || ix[2] < 0 || ix[0] >= nv || ix[1] >= nv || ix[2] >= nv) continue;
    double g[3];
    for (int k = 0; k < 3; ++k) g[k] = (vert(ix[0], k) + vert(ix[1], k) + vert(ix[2], k)) / 3.0;
    for (int j = 0; j < 3; ++j) {
      double d2 = 0.0;
      for (int k = 0; k < 3; ++k) d2 += (vert(ix[j], k) - g[k]) * (vert(ix[j], k) - g[k]);
      rho2 = std::max(rho2, d2);
    }
  }
  *q_limit = rho2 > 0.0 ? kPhaseMax32 / std::sqrt(rho2) : std::numeric_limits<double>::infinity();
  return PFT_OK;
}

pft_status pft_strip_order(const int32_t* tris, int64_t nf, int64_t nv, int32_t* order, uint8_t* meta) {
  if (nf < 0 || nv < 0) return fail(PFT_EINVAL, "negative count");
  if (nf > INT32_MAX / 3 || nv > INT32_MAX) return fail(PFT_EINVAL, "mesh too large for 32-bit indices");
  if (nf > 0 && (tris == nullptr || order == nullptr || meta == nullptr))
    return fail(PFT_EINVAL, "tris, order or meta is NULL");
  if (nf == 0) return PFT_OK;
  // half-edges of the valid faces keyed by their unordered vertex pair; faces that list the same
  // pair (in either direction) share that edge
  auto valid = [&](int64_t f) {
    const int32_t a = tris[3 * f], b = tris[3 * f + 1], c = tris[3 * f + 2];
    return a >= 0 && b >= 0 && c >= 0 && a < nv && b < nv && c < nv && a != b && b != c && c != a;
  };
  std::vector<std::pair<uint64_t, int64_t>> he;
  he.reserve((size_t)nf * 3);
  for (int64_t f = 0; f < nf; ++f) {
    if (!valid(f)) continue;
    for (int e = 0; e < 3; ++e) {
      const uint64_t x = (uint32_t)tris[3 * f + e], y = (uint32_t)tris[3 * f + (e + 1) % 3];
      he.emplace_back(x < y ? (x << 32) | y : (y << 32) | x, 3 * f + e);
    }
  }
  std::sort(he.begin(), he.end());
  // each half-edge points at another half-edge of the same pair (the next one, cyclically)
  std::vector<int64_t> nbr((size_t)nf * 3, -1);
  for (size_t i = 0; i < he.size();) {
    size_t j = i;
    while (j < he.size() && he[j].first == he[i].first) ++j;
    if (j - i > 1)
      for (size_t k = i; k < j; ++k) nbr[he[k].second] = he[k + 1 < j ? k + 1 : i].second;
    i = j;
  }
  // greedy chains: from the last face placed, continue across its edge 1 or 2 (after its rotation) to a
  // face not yet placed, rotated so that the shared edge becomes its edge 0. Leaving through edge 2, the
  // face placed last is marked reflected: its traversal (b, a, c) keeps edge 0 and makes the old edge 2
  // its edge 1, so that the edge a face passes on is always its edge 1.
  std::vector<char> placed((size_t)nf, 0);
  int64_t n = 0;
  for (int64_t f0 = 0; f0 < nf; ++f0) {
    if (placed[f0]) continue;
    int64_t cur = f0;
    int rot = 0;
    placed[cur] = 1;
    order[n] = (int32_t)cur;
    meta[n] = 0;
    ++n;
    for (;;) {
      int64_t next = -1;
      int nrot = 0, via = 0;
      for (int k = 1; k <= 2 && next < 0; ++k) {
        const int64_t slot = 3 * cur + (rot + k) % 3;
        for (int64_t p = nbr[slot]; p >= 0 && p != slot; p = nbr[p]) {
          if (!placed[p / 3]) {
            next = p / 3;
            nrot = (int)(p % 3);
            via = k;
            break;
          }
        }
      }
      if (next < 0) break;
      if (via == 2) meta[n - 1] = (uint8_t)(meta[n - 1] | kMetaReflect);
      placed[next] = 1;
      order[n] = (int32_t)next;
      meta[n] = (uint8_t)(nrot | kMetaLink);
      ++n;
      cur = next;
      rot = nrot;
    }
  }
  return PFT_OK;
}

pft_status pft_forward_3d_poly(const void* verts, pft_dtype vdtype, int64_t nv, const int64_t* face_offsets,
                               const int32_t* face_verts, int64_t nf, const void* q, pft_dtype qdtype, int64_t nq,
                               pft_mode mode, void* out, void* intensity, void* stream) {
  pft_status st = check_mesh_args(verts, vdtype, nv, nullptr, 0, q, qdtype, nq, mode);
  if (st != PFT_OK) return st;
  if (nf < 0) return fail(PFT_EINVAL, "negative count");
  if (nf > INT32_MAX) return fail(PFT_EINVAL, "too many faces");
  if ((st = check_offsets(face_offsets, nf, "face_offsets")) != PFT_OK) return st;
  for (int64_t i = 0; i < nf; ++i) {
    const int64_t n = face_offsets[i + 1] - face_offsets[i];
    if (n < 3 || n > kTileV) return fail(PFT_EINVAL, "each face needs 3 .. 256 vertices");
  }
  const int64_t nref = face_offsets[nf];
  if (nref > INT32_MAX) return fail(PFT_EINVAL, "too many face vertex references");
  if (nref > 0 && face_verts == nullptr) return fail(PFT_EINVAL, "face_verts is NULL");
  if (face_verts && !aligned(face_verts, 4)) return fail(PFT_EINVAL, "face_verts misaligned");
  const bool c128 = mode == PFT_FP64;
  if (nq > 0 && out == nullptr) return fail(PFT_EINVAL, "out is NULL");
  if (out && !aligned(out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "out misaligned");
  if (intensity && !aligned(intensity, c128 ? 8 : 4)) return fail(PFT_EINVAL, "intensity misaligned");
  if (nq == 0) return PFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  // tiles of consecutive faces: at most kTileFP faces and kTileV vertex records each
  std::vector<PolyTile> tiles;
  for (int64_t f = 0; f < nf;) {
    PolyTile t;
    t.f0 = (int32_t)f;
    t.v0 = (int32_t)face_offsets[f];
    while (f < nf && f - t.f0 < kTileFP && face_offsets[f + 1] - t.v0 <= kTileV) ++f;
    t.f1 = (int32_t)f;
    t.v1 = (int32_t)face_offsets[f];
    tiles.push_back(t);
  }
  const int64_t ntiles = (int64_t)tiles.size();
  Arena ar(s);
  MeshInfo* info = ar.get<MeshInfo>(1);
  int64_t* d_off = ar.get<int64_t>(nf + 1);
  FaceP64* f64 = ar.get<FaceP64>(std::max<int64_t>(nf, 1));
  VtxP64* v64 = ar.get<VtxP64>(std::max<int64_t>(nref, 1));
  FaceP32* f32 = c128 ? nullptr : ar.get<FaceP32>(std::max<int64_t>(nf, 1));
  VtxP32* v32 = c128 ? nullptr : ar.get<VtxP32>(std::max<int64_t>(nref, 1));
  const int64_t qblocks = cdiv(nq, (int64_t)kBlock * (c128 ? 1 : kQPTPoly));
  const int64_t sp = std::max<int64_t>(1, std::min<int64_t>(cdiv(kTargetBlocks, qblocks), ntiles));
  const int64_t per = std::max<int64_t>(1, cdiv(ntiles, sp));
  const int splits = (int)std::max<int64_t>(1, cdiv(ntiles, per));
  double2* partial = ar.get<double2>((size_t)splits * nq);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  PolyTile* d_tiles = nullptr;
  if ((st = upload(ar, tiles, &d_tiles, s)) != PFT_OK) return st;
  hipError_t e = hipMemcpyAsync(d_off, face_offsets, sizeof(int64_t) * (nf + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_mesh_info_single(verts, vdtype, 3, nv, info, s);
  if (e == hipSuccess)
    e = launch_poly_records(verts, vdtype, nv, d_off, face_verts, nf, info, c128 ? kTauF64 : kTauF32, f64, v64, s);
  if (e == hipSuccess && !c128) e = launch_poly_records32(f64, v64, nf, kTauRel32, f32, v32, s);
  if (e != hipSuccess) return hip_fail(e, "polygon prologue");
  uint32_t* perm = nullptr;
  if ((st = build_qorder(ar, q, qdtype, nq, nullptr, 1, &perm, s)) != PFT_OK) return st;
  FwdArgs a;
  a.f64 = nullptr;
  a.f32 = nullptr;
  a.info = info;
  a.nf = nf;
  a.q = q;
  a.qdtype = qdtype;
  a.nq = nq;
  a.perm = perm;
  a.splits = splits;
  a.faces_per_split = 0;
  a.split_face = nullptr;
  a.partial = partial;
  a.out = out;
  a.intensity = intensity;
  a.tau0 = c128 ? kTau0F64 : kTau0F32;
  PolyArgs pa;
  pa.f64 = f64;
  pa.v64 = v64;
  pa.f32 = f32;
  pa.v32 = v32;
  pa.tiles = d_tiles;
  pa.ntiles = ntiles;
  pa.tiles_per_split = per;
  const char* nm = c128 ? "fwdpoly_fp64" : "fwdpoly_fp32c";
  prof_begin(nm, s);
  e = c128 ? launch_fwdpoly_fp64(a, pa, s) : launch_fwdpoly_fp32c(a, pa, s);
  prof_end(nm, s);
  if (e != hipSuccess) return hip_fail(e, "polygon transform");
  e = launch_fwd3d_finish(a, c128 ? 1 : 0, s);
  return e == hipSuccess ? PFT_OK : hip_fail(e, "3D finish");
}

pft_status pft_orientation_average(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                   const double* qabs, int64_t nqa, const double* dirs, const double* weights,
                                   int64_t ndir, pft_mode mode, double* out, const int32_t* face_order,
                                   const uint8_t* face_meta, void* stream) {
  pft_status st = check_mesh_args(verts, vdtype, nv, tris, nf, nullptr, PFT_F64, 0, mode);
  if (st != PFT_OK) return st;
  if ((face_order == nullptr) != (face_meta == nullptr)) return fail(PFT_EINVAL, "face_order and face_meta go together");
  if (face_order && !aligned(face_order, 4)) return fail(PFT_EINVAL, "face_order misaligned");
  if (nqa < 0 || ndir < 0) return fail(PFT_EINVAL, "negative count");
  if (nqa > 0 && (qabs == nullptr || out == nullptr)) return fail(PFT_EINVAL, "qabs or out is NULL");
  if (ndir > 0 && (dirs == nullptr || weights == nullptr)) return fail(PFT_EINVAL, "dirs or weights is NULL");
  if ((qabs && !aligned(qabs, 8)) || (dirs && !aligned(dirs, 8)) || (weights && !aligned(weights, 8)) ||
      (out && !aligned(out, 8)))
    return fail(PFT_EINVAL, "argument misaligned");
  if (ndir > 0 && nqa > INT64_MAX / 3 / ndir) return fail(PFT_EINVAL, "nqa * ndir too large");
  if (nqa > INT32_MAX) return fail(PFT_EINVAL, "too many magnitudes");
  if (nqa == 0) return PFT_OK;
  if ((st = strict_mesh(verts, vdtype, nv, tris, nf, nullptr, 0, stream)) != PFT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  if (ndir == 0) {  // empty quadrature: the sum is 0
    hipError_t e = zero_bytes(out, (size_t)nqa * sizeof(double), s);
    return e == hipSuccess ? PFT_OK : hip_fail(e, "zero out");
  }
  const bool c128 = mode == PFT_FP64;
  const int64_t nq = nqa * ndir;
  Arena ar(s);
  double* Q = ar.get<double>((size_t)nq * 3);
  void* I = c128 ? (void*)ar.get<double>(nq) : (void*)ar.get<float>(nq);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  hipError_t e = launch_qdirs(qabs, nqa, dirs, ndir, Q, s);
  if (e != hipSuccess) return hip_fail(e, "orientation Q list");
  st = forward3d_core(ar, verts, vdtype, nv, tris, nf, Q, PFT_F64, nq, mode, nullptr, I, s,
                      nf > 0 ? face_order : nullptr, nf > 0 ? face_meta : nullptr);
  if (st != PFT_OK) return st;
  prof_begin("orient_sum", s);
  e = launch_dir_sum(I, c128 ? PFT_F64 : PFT_F32, weights, nqa, ndir, out, s);
  prof_end("orient_sum", s);
  return e == hipSuccess ? PFT_OK : hip_fail(e, "orientation sum");
}

static pft_status backward3d_impl(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                  const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, const void* grad_out,
                                  void* grad_verts, const uint32_t* q_order, void* stream) {
  pft_status st = check_mesh_args(verts, vdtype, nv, tris, nf, q, qdtype, nq, mode);
  if (st != PFT_OK) return st;
  if (q_order && !aligned(q_order, 4)) return fail(PFT_EINVAL, "q_order misaligned");
  const bool c128 = mode == PFT_FP64;
  if (nq > 0 && grad_out == nullptr) return fail(PFT_EINVAL, "grad_out is NULL");
  if (nv > 0 && grad_verts == nullptr) return fail(PFT_EINVAL, "grad_verts is NULL");
  if (grad_out && !aligned(grad_out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "grad_out misaligned");
  if (grad_verts && !aligned(grad_verts, real_size(vdtype))) return fail(PFT_EINVAL, "grad_verts misaligned");
  if (nv == 0) return PFT_OK;
  if ((st = strict_mesh(verts, vdtype, nv, tris, nf, nullptr, 0, stream)) != PFT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  if (nq == 0 || nf == 0) {
    hipError_t e = zero_bytes(grad_verts, (size_t)nv * 3 * real_size(vdtype), s);
    return e == hipSuccess ? PFT_OK : hip_fail(e, "zero grad");
  }
  Arena ar(s);
  MeshInfo* info = ar.get<MeshInfo>(1);
  Face64* f64 = ar.get<Face64>(nf);
  Face32B* f32 = c128 ? nullptr : ar.get<Face32B>(nf);
  double* gram = c128 ? ar.get<double>((size_t)nf * 8) : nullptr;
  int qs;
  int64_t qper;
  choose_q_splits(nq, nf, c128 ? kTileFB : kTileFB32, &qs, &qper);
  double* partial = ar.get<double>((size_t)qs * nf * 3);
  double* contrib = ar.get<double>((size_t)nf * 9);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  hipError_t e = launch_mesh_info_single(verts, vdtype, 3, nv, info, s);
  if (e == hipSuccess) e = launch_face64(verts, vdtype, nv, tris, nf, info, kTauF64, f64, s);
  if (e == hipSuccess && !c128) e = launch_face32b(f64, nf, kTauB32, kTauRelB32, f32, s);
  if (e == hipSuccess && c128) e = launch_gram64(f64, nf, gram, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint prologue");
  QRec32* rec = nullptr;
  QRec64* rec64 = nullptr;
  if (q_order) {
    uint32_t* perm = nullptr;
    if ((st = caller_qorder(ar, q_order, nq, &perm, s)) != PFT_OK) return st;
    st = qrecs_from_perm(ar, mode, q, qdtype, grad_out, nq, info, nullptr, 1, perm, &rec, &rec64, s);
  } else {
    st = build_qrecs(ar, mode, q, qdtype, grad_out, nq, info, nullptr, 1, &rec, &rec64, s);
  }
  if (st != PFT_OK) return st;
  BwdArgs a;
  a.info = info;
  a.f64 = f64;
  a.f32 = f32;
  a.nf = nf;
  a.q = q;
  a.qdtype = qdtype;
  a.nq = nq;
  a.grad_out = grad_out;
  a.rec = rec;
  a.rec64 = rec64;
  a.qsplits = qs;
  a.q_per_split = qper;
  a.partial = partial;
  const char* nm = main_name(false, mode);
  prof_begin(nm, s);
  e = c128 ? launch_bwd3d_fp64(a, gram, s) : launch_bwd3d_fp32c(a, s);
  prof_end(nm, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint");
  e = launch_bwd_face_contrib(partial, qs, f64, nullptr, nf, contrib, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint reduce");
  return gather_tail(ar, tris, nf, nullptr, nullptr, nv, contrib, grad_verts, vdtype, s);
}

pft_status pft_backward_3d(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                           const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, const void* grad_out,
                           void* grad_verts, void* stream) {
  return backward3d_impl(verts, vdtype, nv, tris, nf, q, qdtype, nq, mode, grad_out, grad_verts, nullptr, stream);
}

pft_status pft_backward_3d_ordered(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                   const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, const void* grad_out,
                                   void* grad_verts, const uint32_t* q_order, void* stream) {
  return backward3d_impl(verts, vdtype, nv, tris, nf, q, qdtype, nq, mode, grad_out, grad_verts, q_order, stream);
}

pft_status pft_intensity_loss_3d(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                 const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, const double* weight,
                                 const double* target, double* loss, void* out, void* grad_verts,
                                 const int32_t* face_order, const uint8_t* face_meta, void* stream) {
  pft_status st = check_mesh_args(verts, vdtype, nv, tris, nf, q, qdtype, nq, mode);
  if (st != PFT_OK) return st;
  const bool c128 = mode == PFT_FP64;
  if (loss == nullptr) return fail(PFT_EINVAL, "loss is NULL");
  if ((face_order == nullptr) != (face_meta == nullptr)) return fail(PFT_EINVAL, "face_order and face_meta go together");
  if (face_order && !aligned(face_order, 4)) return fail(PFT_EINVAL, "face_order misaligned");
  if (nq > 0 && target == nullptr) return fail(PFT_EINVAL, "target is NULL");
  if (!aligned(loss, 8) || (target && !aligned(target, 8)) || (weight && !aligned(weight, 8)))
    return fail(PFT_EINVAL, "loss, target or weight misaligned");
  if (out && !aligned(out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "out misaligned");
  if (grad_verts && !aligned(grad_verts, real_size(vdtype))) return fail(PFT_EINVAL, "grad_verts misaligned");
  if ((st = strict_mesh(verts, vdtype, nv, tris, nf, nullptr, 0, stream)) != PFT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  hipError_t e = hipSuccess;
  if (nq == 0) {  // no Q: L = 0 and no gradient
    e = zero_bytes(loss, sizeof(double), s);
    if (e == hipSuccess && grad_verts && nv > 0) e = zero_bytes(grad_verts, (size_t)nv * 3 * real_size(vdtype), s);
    return e == hipSuccess ? PFT_OK : hip_fail(e, "zero outputs");
  }
  Arena ar(s);
  // shared prologue: one set of face records and one Q order for the forward and the adjoint (with an
  // edge-sharing order the FP32C forward gets its own records in that order)
  const bool ordered = face_order != nullptr && !c128 && nf > 0;
  MeshInfo* info = ar.get<MeshInfo>(1);
  Face64* f64 = ar.get<Face64>(std::max<int64_t>(nf, 1));
  Face64* f64o = ordered ? ar.get<Face64>(nf) : f64;
  Face32* f32 = c128 ? nullptr : ar.get<Face32>(std::max<int64_t>(nf, 1));
  FwdArgs a;
  double2* partial = ar.get<double2>((size_t)plan_forward(nq, nf, c128, -1, a));
  QRec32* rec = c128 ? nullptr : ar.get<QRec32>(nq);
  QRec64* rec64 = c128 ? ar.get<QRec64>(nq) : nullptr;
  double* loss_part = ar.get<double>(loss_blocks(nq));
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  e = launch_mesh_info_single(verts, vdtype, 3, nv, info, s);
  // binary64 records with the binary64 series threshold (the FP32C forward takes its own from Face32)
  if (e == hipSuccess) e = launch_face64(verts, vdtype, nv, tris, nf, info, kTauF64, f64, s);
  if (e == hipSuccess && ordered)
    e = launch_face64(verts, vdtype, nv, tris, nf, info, kTauF64, f64o, s, face_order, face_meta);
  if (e == hipSuccess && !c128) e = launch_face32(f64o, nf, kTauF32, kTauRel32, f32, s);
  if (e != hipSuccess) return hip_fail(e, "loss prologue");
  uint32_t* perm = nullptr;
  if ((st = build_qorder(ar, q, qdtype, nq, nullptr, 1, &perm, s)) != PFT_OK) return st;
  a.f64 = f64o;
  a.f32 = f32;
  a.info = info;
  a.nf = nf;
  a.q = q;
  a.qdtype = qdtype;
  a.nq = nq;
  a.perm = perm;
  a.split_face = nullptr;
  a.partial = partial;
  a.out = out;
  a.intensity = nullptr;
  a.tau0 = c128 ? kTau0F64 : kTau0F32;
  a.share_edges = ordered ? 1 : 0;
  const char* nm = main_name(true, mode);
  prof_begin(nm, s);
  e = c128 ? launch_fwd3d_fp64(a, s) : launch_fwd3d_fp32c(a, s);
  prof_end(nm, s);
  if (e != hipSuccess) return hip_fail(e, "3D transform");
  e = launch_loss_finish(a, weight, target, c128 ? 1 : 0, rec, rec64, loss_part, loss, s);
  if (e != hipSuccess) return hip_fail(e, "loss finish");
  if (!grad_verts || nv == 0) return PFT_OK;
  if (nf == 0) {
    e = zero_bytes(grad_verts, (size_t)nv * 3 * real_size(vdtype), s);
    return e == hipSuccess ? PFT_OK : hip_fail(e, "zero grad");
  }
  Face32B* f32b = c128 ? nullptr : ar.get<Face32B>(nf);
  double* gram = c128 ? ar.get<double>((size_t)nf * 8) : nullptr;
  int qs;
  int64_t qper;
  choose_q_splits(nq, nf, c128 ? kTileFB : kTileFB32, &qs, &qper);
  double* bpart = ar.get<double>((size_t)qs * nf * 3);
  double* contrib = ar.get<double>((size_t)nf * 9);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  e = c128 ? launch_gram64(f64, nf, gram, s) : launch_face32b(f64, nf, kTauB32, kTauRelB32, f32b, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint prologue");
  BwdArgs b;
  b.info = info;
  b.f64 = f64;
  b.f32 = f32b;
  b.nf = nf;
  b.q = q;
  b.qdtype = qdtype;
  b.nq = nq;
  b.grad_out = nullptr;
  b.rec = rec;
  b.rec64 = rec64;
  b.qsplits = qs;
  b.q_per_split = qper;
  b.partial = bpart;
  nm = main_name(false, mode);
  prof_begin(nm, s);
  e = c128 ? launch_bwd3d_fp64(b, gram, s) : launch_bwd3d_fp32c(b, s);
  prof_end(nm, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint");
  e = launch_bwd_face_contrib(bpart, qs, f64, nullptr, nf, contrib, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint reduce");
  return gather_tail(ar, tris, nf, nullptr, nullptr, nv, contrib, grad_verts, vdtype, s);
}

pft_status pft_forward_3d_regions(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                  const int64_t* region_offsets, int64_t nreg, const double* rho, const void* q,
                                  pft_dtype qdtype, int64_t nq, pft_mode mode, void* out, void* out_regions,
                                  void* intensity, const int32_t* face_order, const uint8_t* face_meta,
                                  void* stream) {
  pft_status st = check_mesh_args(verts, vdtype, nv, tris, nf, q, qdtype, nq, mode);
  if (st != PFT_OK) return st;
  if ((st = check_regions(region_offsets, nreg, nf, rho)) != PFT_OK) return st;
  if ((face_order == nullptr) != (face_meta == nullptr)) return fail(PFT_EINVAL, "face_order and face_meta go together");
  if (face_order && !aligned(face_order, 4)) return fail(PFT_EINVAL, "face_order misaligned");
  const bool c128 = mode == PFT_FP64;
  if (nq > 0 && out == nullptr) return fail(PFT_EINVAL, "out is NULL");
  if (out && !aligned(out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "out misaligned");
  if (out_regions && !aligned(out_regions, c128 ? 16 : 8)) return fail(PFT_EINVAL, "out_regions misaligned");
  if (intensity && !aligned(intensity, c128 ? 8 : 4)) return fail(PFT_EINVAL, "intensity misaligned");
  if (nq == 0) return PFT_OK;
  if ((st = strict_mesh(verts, vdtype, nv, tris, nf, region_offsets, nreg, stream)) != PFT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  Arena ar(s);
  RegionPlan plan;
  if ((st = plan_regions(ar, region_offsets, nreg, nq, c128 ? kBlock : fwd_qtile(fwd_qpt(nq)),
                           c128 ? kMinFacesPerSplit : kMinFacesPerSplit * kFwdSplitWaves,
                           c128 ? kTargetBlocks : kTargetBlocksF32, plan, s)) != PFT_OK) return st;
  MeshInfo* info = ar.get<MeshInfo>(1);
  Face64* f64 = ar.get<Face64>(std::max<int64_t>(nf, 1));
  Face32* f32 = c128 ? nullptr : ar.get<Face32>(std::max<int64_t>(nf, 1));
  double2* partial = ar.get<double2>((size_t)std::max(plan.splits, 1) * nq);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  hipError_t e = launch_mesh_info_single(verts, vdtype, 3, nv, info, s);
  const bool ordered = face_order != nullptr && !c128 && nf > 0;
  if (e == hipSuccess)
    e = launch_face64(verts, vdtype, nv, tris, nf, info, c128 ? kTauF64 : kTauF32, f64, s,
                      ordered ? face_order : nullptr, ordered ? face_meta : nullptr);
  if (e == hipSuccess && !c128) e = launch_face32(f64, nf, kTauF32, kTauRel32, f32, s);
  if (e != hipSuccess) return hip_fail(e, "3D prologue");
  double* region_R = nullptr;
  double4* split_geo = nullptr;
  if ((st = region_radii(ar, region_offsets, nreg, f64, plan.d_region_split, plan.splits, &region_R, &split_geo, s)) !=
      PFT_OK)
    return st;
  uint32_t* perm = nullptr;
  if ((st = build_qorder(ar, q, qdtype, nq, nullptr, 1, &perm, s)) != PFT_OK) return st;
  FwdArgs a;
  a.f64 = f64;
  a.f32 = f32;
  a.info = info;
  a.nf = nf;
  a.q = q;
  a.qdtype = qdtype;
  a.nq = nq;
  a.perm = perm;
  a.splits = plan.splits;
  a.faces_per_split = 0;
  a.split_face = plan.d_split_face;
  a.partial = partial;
  a.out = out;
  a.intensity = intensity;
  a.tau0 = c128 ? kTau0F64 : kTauRegion32;
  a.share_edges = ordered ? 1 : 0;
  a.qpt = fwd_qpt(nq);  // as in plan_regions' Q-tile
  a.split_geo = split_geo;
  if (plan.splits > 0) {
    const char* nm = main_name(true, mode);
    prof_begin(nm, s);
    e = c128 ? launch_fwd3d_fp64(a, s) : launch_fwd3d_fp32c(a, s);
    prof_end(nm, s);
    if (e != hipSuccess) return hip_fail(e, "3D transform");
  }
  RegionArgs r;
  r.region_split = plan.d_region_split;
  r.nreg = (int)nreg;
  r.rho = rho;
  r.out_regions = out_regions;
  r.grad_out = nullptr;
  r.rho_part = nullptr;
  r.region_R = region_R;
  e = launch_regions_finish(a, r, c128 ? 1 : 0, s);
  return e == hipSuccess ? PFT_OK : hip_fail(e, "regions finish");
}

pft_status pft_backward_3d_regions(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                   const int64_t* region_offsets, int64_t nreg, const double* rho, const void* q,
                                   pft_dtype qdtype, int64_t nq, pft_mode mode, const void* grad_out,
                                   void* grad_verts, double* grad_rho, void* grad_q, void* stream) {
  pft_status st = check_mesh_args(verts, vdtype, nv, tris, nf, q, qdtype, nq, mode);
  if (st != PFT_OK) return st;
  if ((st = check_regions(region_offsets, nreg, nf, rho)) != PFT_OK) return st;
  const bool c128 = mode == PFT_FP64;
  if (nq > 0 && grad_out == nullptr) return fail(PFT_EINVAL, "grad_out is NULL");
  if (grad_out && !aligned(grad_out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "grad_out misaligned");
  if (grad_verts && !aligned(grad_verts, real_size(vdtype))) return fail(PFT_EINVAL, "grad_verts misaligned");
  if (grad_rho && !aligned(grad_rho, 8)) return fail(PFT_EINVAL, "grad_rho misaligned");
  if (grad_q && !aligned(grad_q, real_size(qdtype))) return fail(PFT_EINVAL, "grad_q misaligned");
  const bool want_v = grad_verts != nullptr && nv > 0;
  const bool want_r = grad_rho != nullptr && nreg > 0;
  const bool want_q = grad_q != nullptr && nq > 0;
  if (!want_v && !want_r && !want_q) return PFT_OK;
  if ((st = strict_mesh(verts, vdtype, nv, tris, nf, region_offsets, nreg, stream)) != PFT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  hipError_t e = hipSuccess;
  if (nq == 0 || nf == 0) {  // no Q or no faces: every gradient is zero
    if (want_v) e = zero_bytes(grad_verts, (size_t)nv * 3 * real_size(vdtype), s);
    if (e == hipSuccess && want_r) e = zero_bytes(grad_rho, (size_t)nreg * sizeof(double), s);
    if (e == hipSuccess && want_q) e = zero_bytes(grad_q, (size_t)nq * 3 * real_size(qdtype), s);
    return e == hipSuccess ? PFT_OK : hip_fail(e, "zero gradients");
  }
  Arena ar(s);
  MeshInfo* info = ar.get<MeshInfo>(1);
  Face64* f64 = ar.get<Face64>(nf);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  e = launch_mesh_info_single(verts, vdtype, 3, nv, info, s);
  if (e == hipSuccess) e = launch_face64(verts, vdtype, nv, tris, nf, info, kTauF64, f64, s);
  if (e != hipSuccess) return hip_fail(e, "regions prologue");
  Face32B* f32b = nullptr;
  double* gram = nullptr;
  if (want_v || want_q) {
    f32b = c128 ? nullptr : ar.get<Face32B>(nf);
    gram = c128 ? ar.get<double>((size_t)nf * 8) : nullptr;
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    e = c128 ? launch_gram64(f64, nf, gram, s) : launch_face32b(f64, nf, kTauB32, kTauRelB32, f32b, s);
    if (e != hipSuccess) return hip_fail(e, "regions prologue");
  }
  // one visiting order of Q for every part below
  uint32_t* perm = nullptr;
  if ((st = build_qorder(ar, q, qdtype, nq, nullptr, 1, &perm, s)) != PFT_OK) return st;
  // dL/dv: the vertex adjoint with each face's partial weighted by its region's density
  if (want_v) {
    int64_t* d_off = nullptr;
    std::vector<int64_t> offv(region_offsets, region_offsets + nreg + 1);
    if ((st = upload(ar, offv, &d_off, s)) != PFT_OK) return st;
    double* face_w = ar.get<double>(nf);
    int qs;
    int64_t qper;
    choose_q_splits(nq, nf, c128 ? kTileFB : kTileFB32, &qs, &qper);
    double* partial = ar.get<double>((size_t)qs * nf * 3);
    double* contrib = ar.get<double>((size_t)nf * 9);
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    e = launch_face_weights(d_off, (int)nreg, rho, nf, face_w, s);
    if (e != hipSuccess) return hip_fail(e, "face weights");
    QRec32* rec = nullptr;
    QRec64* rec64 = nullptr;
    if ((st = qrecs_from_perm(ar, mode, q, qdtype, grad_out, nq, info, nullptr, 1, perm, &rec, &rec64, s)) != PFT_OK)
      return st;
    BwdArgs b;
    b.info = info;
    b.f64 = f64;
    b.f32 = f32b;
    b.nf = nf;
    b.q = q;
    b.qdtype = qdtype;
    b.nq = nq;
    b.grad_out = grad_out;
    b.rec = rec;
    b.rec64 = rec64;
    b.qsplits = qs;
    b.q_per_split = qper;
    b.partial = partial;
    const char* nm = main_name(false, mode);
    prof_begin(nm, s);
    e = c128 ? launch_bwd3d_fp64(b, gram, s) : launch_bwd3d_fp32c(b, s);
    prof_end(nm, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint");
    e = launch_bwd_face_contrib(partial, qs, f64, face_w, nf, contrib, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint reduce");
    if ((st = gather_tail(ar, tris, nf, nullptr, nullptr, nv, contrib, grad_verts, vdtype, s)) != PFT_OK) return st;
  }
  if (!want_r && !want_q) return PFT_OK;
  const int64_t nblocks = finish_blocks(nq);
  double* rho_part = want_r ? ar.get<double>((size_t)nblocks * nreg) : nullptr;
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  RegionArgs r;
  r.region_R = nullptr;
  r.nreg = (int)nreg;
  r.rho = rho;
  r.out_regions = nullptr;
  r.grad_out = grad_out;
  r.rho_part = rho_part;
  if (want_q) {
    // dL/dQ (and dL/drho from the same partials): the grad_Q kernel
    RegionPlan plan;
    if ((st = plan_regions(ar, region_offsets, nreg, nq, c128 ? kBlock : (int64_t)kBlock * kQPTDQ, kMinFacesPerSplit,
                             kTargetBlocks, plan, s)) != PFT_OK) return st;
    double2* partial = ar.get<double2>((size_t)std::max(plan.splits, 1) * 4 * nq);
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    DqArgs d;
    d.info = info;
    d.f64 = f64;
    d.gram = gram;
    d.f32 = f32b;
    d.nf = nf;
    d.q = q;
    d.qdtype = qdtype;
    d.nq = nq;
    d.perm = perm;
    d.splits = plan.splits;
    d.faces_per_split = 0;
    d.split_face = plan.d_split_face;
    d.partial = partial;
    d.tau = c128 ? kTauDQ : kTauRegion32;
    double* region_R = nullptr;
    double4* split_geo = nullptr;
    if ((st = region_radii(ar, region_offsets, nreg, f64, plan.d_region_split, plan.splits, &region_R, &split_geo, s)) !=
        PFT_OK)
      return st;
    d.split_geo = split_geo;
    r.region_R = region_R;
    const char* nm = c128 ? "dq3d_fp64" : "dq3d_fp32c";
    prof_begin(nm, s);
    e = c128 ? launch_dq3d_fp64(d, s) : launch_dq3d_fp32c(d, s);
    prof_end(nm, s);
    if (e != hipSuccess) return hip_fail(e, "grad_Q transform");
    r.region_split = plan.d_region_split;
    e = launch_dq_finish(d, r, c128 ? 1 : 0, grad_q, qdtype, s);
    if (e != hipSuccess) return hip_fail(e, "grad_Q finish");
  } else {
    // dL/drho only: the forward's partials per region
    RegionPlan plan;
    if ((st = plan_regions(ar, region_offsets, nreg, nq, c128 ? kBlock : fwd_qtile(fwd_qpt(nq)),
                           c128 ? kMinFacesPerSplit : kMinFacesPerSplit * kFwdSplitWaves,
                           c128 ? kTargetBlocks : kTargetBlocksF32, plan, s)) != PFT_OK) return st;
    Face32* f32 = c128 ? nullptr : ar.get<Face32>(nf);
    double2* partial = ar.get<double2>((size_t)std::max(plan.splits, 1) * nq);
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    if (!c128) {
      e = launch_face32(f64, nf, kTauF32, kTauRel32, f32, s);
      if (e != hipSuccess) return hip_fail(e, "regions prologue");
    }
    FwdArgs a;
    a.f64 = f64;
    a.f32 = f32;
    a.info = info;
    a.nf = nf;
    a.q = q;
    a.qdtype = qdtype;
    a.nq = nq;
    a.perm = perm;
    a.splits = plan.splits;
    a.faces_per_split = 0;
    a.split_face = plan.d_split_face;
    a.partial = partial;
    a.out = nullptr;
    a.intensity = nullptr;
    a.tau0 = c128 ? kTau0F64 : kTauRegion32;
    a.qpt = fwd_qpt(nq);  // as in plan_regions' Q-tile
    double* region_R = nullptr;
    double4* split_geo = nullptr;
    if ((st = region_radii(ar, region_offsets, nreg, f64, plan.d_region_split, plan.splits, &region_R, &split_geo, s)) !=
        PFT_OK)
      return st;
    a.split_geo = split_geo;
    r.region_R = region_R;
    if (plan.splits > 0) {
      const char* nm = main_name(true, mode);
      prof_begin(nm, s);
      e = c128 ? launch_fwd3d_fp64(a, s) : launch_fwd3d_fp32c(a, s);
      prof_end(nm, s);
      if (e != hipSuccess) return hip_fail(e, "3D transform");
    }
    r.region_split = plan.d_region_split;
    e = launch_regions_finish(a, r, c128 ? 1 : 0, s);
    if (e != hipSuccess) return hip_fail(e, "regions finish");
  }
  if (want_r) {
    e = launch_rho_reduce(rho_part, nblocks, (int)nreg, grad_rho, s);
    if (e != hipSuccess) return hip_fail(e, "rho reduce");
  }
  return PFT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched entry points
// ---------------------------------------------------------------------------
namespace {

struct BatchPrep {
  int64_t n = 0, nv = 0, nf = 0, nq = 0;
  int64_t* d_vert_off = nullptr;
  int64_t* d_tri_off = nullptr;
  int64_t* d_q_off = nullptr;
  int32_t* d_face_mesh = nullptr;
  MeshInfo* info = nullptr;
  Face64* f64 = nullptr;
};

pft_status check_batch(const pft_mesh_batch* b, int mode) {
  if (!b) return fail(PFT_EINVAL, "batch is NULL");
  if (b->n_meshes < 0) return fail(PFT_EINVAL, "negative mesh count");
  if (b->n_meshes > INT32_MAX) return fail(PFT_EINVAL, "too many meshes");
  pft_status st = check_offsets(b->vert_offsets, b->n_meshes, "vert_offsets");
  if (st == PFT_OK) st = check_offsets(b->tri_offsets, b->n_meshes, "tri_offsets");
  if (st == PFT_OK) st = check_offsets(b->q_offsets, b->n_meshes, "q_offsets");
  if (st != PFT_OK) return st;
  const int64_t n = b->n_meshes;
  return check_mesh_args(b->verts, b->vdtype, b->vert_offsets[n], b->tris, b->tri_offsets[n], b->q, b->qdtype,
                         b->q_offsets[n], mode);
}

pft_status batch_prologue(Arena& ar, const pft_mesh_batch* b, double tau, BatchPrep& p, hipStream_t s,
                          const int32_t* order = nullptr, const uint8_t* meta = nullptr) {
  p.n = b->n_meshes;
  p.nv = b->vert_offsets[p.n];
  p.nf = b->tri_offsets[p.n];
  p.nq = b->q_offsets[p.n];
  p.d_vert_off = ar.get<int64_t>(p.n + 1);
  p.d_tri_off = ar.get<int64_t>(p.n + 1);
  p.d_q_off = ar.get<int64_t>(p.n + 1);
  p.d_face_mesh = ar.get<int32_t>(std::max<int64_t>(p.nf, 1));
  p.info = ar.get<MeshInfo>(std::max<int64_t>(p.n, 1));
  p.f64 = ar.get<Face64>(std::max<int64_t>(p.nf, 1));
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  const size_t ob = sizeof(int64_t) * (p.n + 1);
  hipError_t e = hipMemcpyAsync(p.d_vert_off, b->vert_offsets, ob, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p.d_tri_off, b->tri_offsets, ob, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p.d_q_off, b->q_offsets, ob, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "offsets upload");
  if (p.n > 0) e = launch_mesh_info(b->verts, b->vdtype, p.d_vert_off, p.n, p.info, s);
  if (e == hipSuccess) e = launch_fill_face_mesh(p.d_tri_off, p.n, p.nf, p.d_face_mesh, s);
  if (e == hipSuccess)
    e = launch_face64_batch(b->verts, b->vdtype, b->tris, p.d_vert_off, p.d_tri_off, p.d_face_mesh, p.nf, p.info,
                            tau, p.f64, s, order, meta);
  if (e != hipSuccess) return hip_fail(e, "batch prologue");
  return PFT_OK;
}


}  // namespace

extern "C" {

static pft_status batch_forward_impl(const pft_mesh_batch* b, pft_mode mode, void* out, void* intensity,
                                     const int32_t* face_order, const uint8_t* face_meta, void* stream) {
  pft_status st = check_batch(b, mode);
  if (st != PFT_OK) return st;
  const bool c128 = mode == PFT_FP64;
  const bool share = face_order != nullptr && !c128;
  if ((face_order == nullptr) != (face_meta == nullptr)) return fail(PFT_EINVAL, "face_order and face_meta go together");
  if (face_order && !aligned(face_order, 4)) return fail(PFT_EINVAL, "face_order misaligned");
  const int64_t n = b->n_meshes, nq_total = b->q_offsets[n];
  if (nq_total > 0 && out == nullptr) return fail(PFT_EINVAL, "out is NULL");
  if (out && !aligned(out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "out misaligned");
  if (intensity && !aligned(intensity, c128 ? 8 : 4)) return fail(PFT_EINVAL, "intensity misaligned");
  if (nq_total == 0) return PFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  Arena ar(s);
  BatchPrep p;
  st = batch_prologue(ar, b, c128 ? kTauF64 : kTauF32, p, s, share ? face_order : nullptr,
                      share ? face_meta : nullptr);
  if (st != PFT_OK) return st;
  Face32* f32 = nullptr;
  if (!c128) {
    f32 = ar.get<Face32>(std::max<int64_t>(p.nf, 1));
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    hipError_t e = launch_face32(p.f64, p.nf, kTauF32, kTauRel32, f32, s);
    if (e != hipSuccess) return hip_fail(e, "batch prologue");
  }
  // work items: (mesh, Q-tile, face chunk), longest first, for given tile sizes; returns the number of
  // partial slots they need
  // The mesh's work items as up to four runs of equal-size items (full or last face chunk x full or last
  // Q-tile), longest items first over all meshes; returns the partial slots and sets n_items.
  auto make_groups = [&](const BatchTiles& t, std::vector<BatchGroupFwd>& groups, std::vector<int64_t>& q_part,
                         std::vector<int32_t>& q_chunks, int64_t& n_items) {
    groups.clear();
    q_part.assign(n, 0);
    q_chunks.assign(n, 1);
    int64_t P = 0;
    const int64_t qtile = c128 ? kBlock : (int64_t)64 * t.qpt;  // Q per item (a block in binary64, a wavefront in FP32C)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t nqi = b->q_offsets[i + 1] - b->q_offsets[i];
      const int64_t nfi = b->tri_offsets[i + 1] - b->tri_offsets[i];
      int64_t C = 1, cf = nfi;
      if (nfi > 0) {
        C = cdiv(nfi, t.chunk_f);
        cf = cdiv(cdiv(nfi, C), kTileF) * kTileF;
        C = cdiv(nfi, cf);
      }
      q_part[i] = P;
      q_chunks[i] = (int32_t)C;
      const int64_t T = cdiv(nqi, qtile);
      // chunks [0, C-1) of cf faces and the last one; Q-tiles [0, T-1) of qtile Q and the last one
      const int64_t last_nf = nfi > 0 ? nfi - (C - 1) * cf : 0, last_nq = nqi - (T - 1) * qtile;
      for (int cl = 0; cl < 2 && T > 0; ++cl) {
        const int64_t c0 = cl == 0 ? 0 : C - 1, nc = cl == 0 ? C - 1 : 1;
        for (int tl = 0; tl < 2; ++tl) {
          const int64_t t0 = tl == 0 ? 0 : T - 1, ntq = tl == 0 ? T - 1 : 1;
          if (nc <= 0 || ntq <= 0) continue;
          BatchGroupFwd g;
          g.first = nc * ntq;  // the group's item count until the prefix pass below
          g.f_base = b->tri_offsets[i] + c0 * cf;
          g.q_base = b->q_offsets[i] + t0 * qtile;
          g.part_base = P + c0 * nqi + t0 * qtile;
          g.part_stride = nqi;
          g.mesh = (int32_t)i;
          g.ntq = (int32_t)ntq;
          g.cf = (int32_t)cf;
          g.qtile = (int32_t)qtile;
          g.nf = (int32_t)(cl == 0 ? cf : last_nf);
          g.nq = (int32_t)(tl == 0 ? qtile : last_nq);
          groups.push_back(g);
        }
      }
      P += C * nqi;
    }
    std::stable_sort(groups.begin(), groups.end(), [](const BatchGroupFwd& x, const BatchGroupFwd& y) {
      return (int64_t)x.nf * x.nq > (int64_t)y.nf * y.nq;
    });
    n_items = 0;
    for (BatchGroupFwd& g : groups) {
      const int64_t cnt = g.first;
      g.first = n_items;
      n_items += cnt;
    }
    return P;
  };
  BatchTiles chosen;
  std::vector<BatchTiles> cands;
  std::string key;
  if (!c128 && autotune_enabled()) {
    double pairs = 0.0;
    for (int64_t i = 0; i < n; ++i)
      pairs += (double)(b->tri_offsets[i + 1] - b->tri_offsets[i]) * (double)(b->q_offsets[i + 1] - b->q_offsets[i]);
    key = tune_key("batch_forward", mode, share, n, pairs, p.nf);
    if (!tuned_tiles(key, &chosen))
      for (int qpt : {1, 2, 3})
        for (int64_t cf : {512, 1024, 2048, 4096}) {
          BatchTiles t;
          t.qpt = qpt;
          t.chunk_f = cf;
          cands.push_back(t);
        }
  }
  std::vector<BatchGroupFwd> groups;
  std::vector<int64_t> q_part;
  std::vector<int32_t> q_chunks;
  int64_t n_items_max = 0;
  {  // keep the partial slots within kBatchPartialCapBytes: longer chunks for the choice, fewer candidates
    int64_t max_nf = 1;
    for (int64_t i = 0; i < n; ++i) max_nf = std::max<int64_t>(max_nf, b->tri_offsets[i + 1] - b->tri_offsets[i]);
    const int64_t cap_slots = kBatchPartialCapBytes / (int64_t)sizeof(double2);
    while (make_groups(chosen, groups, q_part, q_chunks, n_items_max) > cap_slots && chosen.chunk_f < max_nf)
      chosen.chunk_f *= 2;
    cands.erase(std::remove_if(cands.begin(), cands.end(),
                               [&](const BatchTiles& t) {
                                 return make_groups(t, groups, q_part, q_chunks, n_items_max) > cap_slots;
                               }),
                cands.end());
  }
  int64_t Pmax = make_groups(chosen, groups, q_part, q_chunks, n_items_max);
  for (const BatchTiles& t : cands) Pmax = std::max(Pmax, make_groups(t, groups, q_part, q_chunks, n_items_max));
  double2* partial = ar.get<double2>(std::max<int64_t>(Pmax, 1));
  uint32_t* counter = ar.get<uint32_t>(1);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  uint32_t* perm = nullptr;
  if ((st = build_qorder(ar, b->q, b->qdtype, nq_total, p.d_q_off, n, &perm, s)) != PFT_OK) return st;
  const double tau0 = c128 ? kTau0F64 : kTau0F32;
  auto run = [&](const BatchTiles& t, bool profile) -> pft_status {
    int64_t n_items = 0;
    make_groups(t, groups, q_part, q_chunks, n_items);
    if (groups.size() > 0x7fffffff || n_items > 0xffffffffLL) return fail(PFT_EINVAL, "too many batch work items");
    BatchGroupFwd* d_groups;
    int64_t* d_q_part;
    int32_t* d_q_chunks;
    pft_status rs;
    if ((rs = upload(ar, groups, &d_groups, s)) != PFT_OK) return rs;
    if ((rs = upload(ar, q_part, &d_q_part, s)) != PFT_OK) return rs;
    if ((rs = upload(ar, q_chunks, &d_q_chunks, s)) != PFT_OK) return rs;
    hipError_t e = launch_zero_u32(counter, 1, s);
    if (e != hipSuccess) return hip_fail(e, "counter reset");
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(n_items, 1),
                                            (int64_t)num_cus() * batch_fwd_blocks_per_cu(mode, share, t.qpt));
    if (profile) prof_begin("batch_fwd", s);
    e = launch_batch_fwd(mode, d_groups, (int)groups.size(), n_items, counter, p.f64, f32, b->q, b->qdtype, perm,
                         partial, p.info, tau0, grid, s, share, t.qpt);
    if (profile) prof_end("batch_fwd", s);
    if (e != hipSuccess) return hip_fail(e, "batch forward");
    e = launch_batch_fwd_finish(partial, p.d_q_off, n, d_q_part, d_q_chunks, p.info, b->q, b->qdtype, perm, nq_total,
                                tau0, c128 ? 1 : 0, out, intensity, s);
    return e == hipSuccess ? PFT_OK : hip_fail(e, "batch finish");
  };
  if (!cands.empty()) {
    std::vector<float> ms;
    const int best = time_candidates((int)cands.size(), [&](int i) { return run(cands[i], false); }, s, ms);
    chosen = cands[best >= 0 ? best : 0];
    std::string log = key + ": qpt=" + std::to_string(chosen.qpt) + " faces/item=" + std::to_string(chosen.chunk_f) +
                      " (candidates qpt x faces/item, ms:";
    for (size_t i = 0; i < cands.size(); ++i)
      log += " " + std::to_string(cands[i].qpt) + "x" + std::to_string(cands[i].chunk_f) + "=" +
             std::to_string(ms[i]).substr(0, 7);
    keep_tiles(key, chosen, log + ")");
  }
  return run(chosen, true);
}

pft_status pft_batch_forward(const pft_mesh_batch* b, pft_mode mode, void* out, void* intensity, void* stream) {
  return batch_forward_impl(b, mode, out, intensity, nullptr, nullptr, stream);
}

pft_status pft_batch_forward_ordered(const pft_mesh_batch* b, const int32_t* face_order, const uint8_t* face_meta,
                                     pft_mode mode, void* out, void* intensity, void* stream) {
  if (b && b->n_meshes > 0 && b->tri_offsets && b->tri_offsets[b->n_meshes] > 0 &&
      (face_order == nullptr || face_meta == nullptr))
    return fail(PFT_EINVAL, "face_order or face_meta is NULL");
  return batch_forward_impl(b, mode, out, intensity, face_order, face_meta, stream);
}

pft_status pft_batch_backward(const pft_mesh_batch* b, pft_mode mode, const void* grad_out, void* grad_verts,
                              void* stream) {
  pft_status st = check_batch(b, mode);
  if (st != PFT_OK) return st;
  const bool c128 = mode == PFT_FP64;
  const int64_t n = b->n_meshes, nv_total = b->vert_offsets[n], nq_total = b->q_offsets[n];
  const int64_t nf_total = b->tri_offsets[n];
  if (nq_total > 0 && grad_out == nullptr) return fail(PFT_EINVAL, "grad_out is NULL");
  if (nv_total > 0 && grad_verts == nullptr) return fail(PFT_EINVAL, "grad_verts is NULL");
  if (grad_out && !aligned(grad_out, c128 ? 16 : 8)) return fail(PFT_EINVAL, "grad_out misaligned");
  if (grad_verts && !aligned(grad_verts, real_size(b->vdtype))) return fail(PFT_EINVAL, "grad_verts misaligned");
  if (nv_total == 0) return PFT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ensure_pool();
  if (nf_total == 0) {
    hipError_t e = zero_bytes(grad_verts, (size_t)nv_total * 3 * real_size(b->vdtype), s);
    return e == hipSuccess ? PFT_OK : hip_fail(e, "zero grad");
  }
  Arena ar(s);
  BatchPrep p;
  st = batch_prologue(ar, b, kTauF64, p, s);
  if (st != PFT_OK) return st;
  Face32B* f32b = nullptr;
  QRec32* rec = nullptr;
  double* gram = nullptr;
  hipError_t e = hipSuccess;
  if (c128) {
    gram = ar.get<double>((size_t)p.nf * 8);
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    e = launch_gram64(p.f64, p.nf, gram, s);
  } else {
    f32b = ar.get<Face32B>(p.nf);
    if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
    e = launch_face32b(p.f64, p.nf, kTauB32, kTauRelB32, f32b, s);
  }
  if (e != hipSuccess) return hip_fail(e, "batch adjoint prologue");
  QRec64* rec64 = nullptr;
  if ((st = build_qrecs(ar, mode, b->q, b->qdtype, grad_out, nq_total, p.info, p.d_q_off, n, &rec, &rec64, s)) !=
      PFT_OK)
    return st;
  const int64_t ftile = c128 ? kTileFB : kTileFB32;  // faces per item (one block)
  // work items: (mesh, face tile, Q chunk), longest first, for a given Q chunk; returns the partial slots
  std::vector<BatchItemBwd> items;
  std::vector<int64_t> face_base;
  std::vector<int32_t> face_nchunks;
  auto make_items = [&](int64_t chunk_q) {
    items.clear();
    face_base.assign(n, 0);
    face_nchunks.assign(n, 1);
    int64_t B = 0;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t nqi = b->q_offsets[i + 1] - b->q_offsets[i];
      const int64_t nfi = b->tri_offsets[i + 1] - b->tri_offsets[i];
      const int64_t S = std::max<int64_t>(1, cdiv(nqi, chunk_q));
      const int64_t cq = std::max<int64_t>(1, cdiv(nqi, S));
      face_base[i] = B;
      face_nchunks[i] = (int32_t)S;
      for (int64_t sc = 0; sc < S; ++sc) {
        for (int64_t ft = 0; ft < nfi; ft += ftile) {
          BatchItemBwd it;
          it.mesh = (int32_t)i;
          it.qchunk = (int32_t)sc;
          it.f0 = b->tri_offsets[i] + ft;
          it.nf = (int32_t)std::min<int64_t>(ftile, nfi - ft);
          it.pad = 0;
          it.q0 = b->q_offsets[i] + std::min(nqi, sc * cq);
          it.nq = std::max<int64_t>(0, std::min(cq, nqi - sc * cq));
          it.part = B + sc * nfi + ft;
          items.push_back(it);
        }
      }
      B += S * nfi;
    }
    std::stable_sort(items.begin(), items.end(), [](const BatchItemBwd& x, const BatchItemBwd& y) {
      return (int64_t)x.nf * x.nq > (int64_t)y.nf * y.nq;
    });
    return B;
  };
  BatchTiles chosen;
  std::vector<int64_t> cands;
  std::string key;
  if (!c128 && autotune_enabled()) {
    double pairs = 0.0;
    for (int64_t i = 0; i < n; ++i)
      pairs += (double)(b->tri_offsets[i + 1] - b->tri_offsets[i]) * (double)(b->q_offsets[i + 1] - b->q_offsets[i]);
    key = tune_key("batch_backward", mode, false, n, pairs, p.nf);
    if (!tuned_tiles(key, &chosen)) cands = {32768, 65536, 131072};
  }
  int64_t Bmax = make_items(chosen.chunk_q);
  for (int64_t cq : cands) Bmax = std::max(Bmax, make_items(cq));
  double* partial = ar.get<double>((size_t)std::max<int64_t>(Bmax, 1) * 3);
  double* contrib = ar.get<double>((size_t)p.nf * 9);
  uint32_t* counter = ar.get<uint32_t>(1);
  if (ar.failed) return fail(PFT_ENOMEM, "temporary allocation failed");
  int32_t* d_face_nchunks = nullptr;
  int64_t* d_face_base = nullptr;
  auto run = [&](int64_t chunk_q, bool profile) -> pft_status {
    make_items(chunk_q);
    BatchItemBwd* d_items;
    pft_status rs;
    if ((rs = upload(ar, items, &d_items, s)) != PFT_OK) return rs;
    if ((rs = upload(ar, face_base, &d_face_base, s)) != PFT_OK) return rs;
    if ((rs = upload(ar, face_nchunks, &d_face_nchunks, s)) != PFT_OK) return rs;
    hipError_t re = launch_zero_u32(counter, 1, s);
    if (re != hipSuccess) return hip_fail(re, "counter reset");
    const int64_t n_items = (int64_t)items.size();
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(n_items, 1),
                                            (int64_t)num_cus() * batch_bwd_blocks_per_cu(mode));
    if (profile) prof_begin("batch_bwd", s);
    re = launch_batch_bwd(mode, d_items, n_items, counter, p.f64, gram, f32b, rec, rec64, partial, grid, s);
    if (profile) prof_end("batch_bwd", s);
    return re == hipSuccess ? PFT_OK : hip_fail(re, "batch adjoint");
  };
  if (!cands.empty()) {
    std::vector<float> ms;
    const int best = time_candidates((int)cands.size(), [&](int i) { return run(cands[i], false); }, s, ms);
    chosen.chunk_q = cands[best >= 0 ? best : 0];
    std::string log = key + ": Q/item=" + std::to_string(chosen.chunk_q) + " (candidates Q/item, ms:";
    for (size_t i = 0; i < cands.size(); ++i)
      log += " " + std::to_string(cands[i]) + "=" + std::to_string(ms[i]).substr(0, 7);
    keep_tiles(key, chosen, log + ")");
  }
  if ((st = run(chosen.chunk_q, true)) != PFT_OK) return st;
  e = launch_batch_bwd_reduce(partial, d_face_base, d_face_nchunks, p.d_tri_off, p.d_face_mesh, p.f64, p.nf, contrib,
                              s);
  if (e != hipSuccess) return hip_fail(e, "batch adjoint reduce");
  return gather_tail(ar, b->tris, p.nf, p.d_vert_off, p.d_face_mesh, nv_total, contrib, grad_verts, b->vdtype, s);
}

}  // extern "C"

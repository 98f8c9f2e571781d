// Serving runtime: HBM-budget admission, continuous chi^2 batching, chunked maps.
//
// One scheduler thread owns all HIP work of the server.  Device memory comes from one arena
// allocated at start (first-fit with coalescing), so admission never calls hipMalloc and the
// budget is a hard bound.  chi^2 requests admitted while a batch is on the device form the
// next batch (one persistent launch per (mode, precision)); map requests are cut into row
// chunks that run on the other streams, so small chi^2 requests are not queued behind large
// maps.  Each chunk's rows are copied to the host right after they are computed.  A map is
// bound to one map stream when its first chunk starts (its chunks stay in order there); a
// free map stream runs the next chunk of the map with the least remaining work among its own
// maps and the unbound ones (shortest remaining first at chunk granularity), so a small
// magnification map overtakes a large singularity map between two of its chunks.
// Completion is detected with events; latencies use the host steady clock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "lf_api_internal.h"
#include "lf_chi2.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Arena {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  bool init(size_t bytes) {
    if (hipMalloc((void**)&base, bytes) != hipSuccess) return false;
    size = bytes;
    free_[0] = bytes;
    return true;
  }
  void* alloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        return base + off;
      }
    }
    return nullptr;
  }
  void release(void* p, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    size_t off = (char*)p - base;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
    }
  }
};

struct Req {
  int64_t id = 0;
  lf_request r{};
  std::vector<double> params;
  Clock::time_point t_submit, t_done;
  int status = 0;                          // 0 pending, 1 done, < 0 error
  bool admitted = false, launched = false;
  std::vector<std::pair<void*, size_t>> blocks;
  // chi^2
  lf::Chi2Args A{};
  double* d_params = nullptr;
  // maps
  lf::MainRec* mains = nullptr;
  lf::MulRec* muls = nullptr;
  lf::MemRec32* m32 = nullptr;
  lf::MemRec64* m64 = nullptr;
  double* d_out = nullptr;
  int* d_flags = nullptr;
  double* part = nullptr;
  int n_planes = 0;
  long long P = 0;
  int next_row = 0;
  int stream = -1;                         // map stream the map is bound to (-1: not started)
  bool expanded = false;
  size_t footprint = 0;
  long long remaining() const { return (long long)(r.grid.ny - next_row) * r.grid.nx * n_planes; }
};

struct Unit {                               // work on the device, awaiting its event
  hipEvent_t ev;
  int stream;
  std::vector<std::shared_ptr<Req>> reqs;
  std::vector<lf::Chi2Args> args;           // host sources of the batch tables, kept alive
  std::vector<lf::BatchTile> tiles;
  std::vector<int> samp;
  std::shared_ptr<Req> map;                 // map chunk: its request
  bool last_chunk = false;
};

constexpr size_t TABLE_BYTES = 8u << 20;    // batch tables of the one chi^2 batch in flight

}  // namespace

struct lf_server {
  lf_ctx* ctx = nullptr;
  lf_serve_config cfg{};
  Arena arena;
  char* tables = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<bool> busy;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  bool stop = false;
  int64_t next_id = 1;
  std::deque<std::shared_ptr<Req>> incoming, pending;
  std::vector<std::shared_ptr<Req>> admitted_chi2, maps_queue;
  std::vector<std::shared_ptr<Req>> map_bound;    // started maps, each bound to one map stream
  std::vector<Unit> inflight;
  std::map<int64_t, std::shared_ptr<Req>> all;
  std::vector<hipEvent_t> ev_pool;
  void loop();
  hipEvent_t ev() {
    if (!ev_pool.empty()) { hipEvent_t e = ev_pool.back(); ev_pool.pop_back(); return e; }
    hipEvent_t e;
    hipEventCreateWithFlags(&e, hipEventDisableTiming);
    return e;
  }
};

namespace {

size_t chi2_footprint(const lf_request& r) {
  size_t S = r.S, n = S * r.cons->n_img;
  return 256 * 13 + sizeof(int) + sizeof(double) * S * r.model->n_free + sizeof(double) * S + sizeof(int) * S +
         sizeof(lf::MainRec) * std::max<size_t>(1, S * r.model->main.size()) + sizeof(lf::MulRec) * S +
         sizeof(double) * n * (5 + 6 + 1 + 1) + sizeof(int) * n * 2 + sizeof(double) * S * r.cons->n_fam * 2;
}
int map_planes(int kind) { return kind == LF_REQ_SING_MAP ? 6 : 1; }
size_t map_footprint(const lf_server* s, const lf_request& r) {
  long long P = (long long)r.grid.nx * r.grid.ny;
  long long chunkP = (long long)s->cfg.map_chunk_rows * r.grid.nx;
  size_t nb = r.model->mem.size();
  const bool dev = r.out_device != nullptr;     // the caller's device memory holds the result
  return 256 * 10 + sizeof(double) * r.model->n_free + (dev ? 0 : sizeof(double) * map_planes(r.kind) * P) +
         (dev && !r.flags_device ? sizeof(int) * chunkP : dev ? 0 : sizeof(int) * P) +
         chunkP * (sizeof(double) * 9 + sizeof(int)) + sizeof(lf::MainRec) * std::max<size_t>(1, r.model->main.size()) +
         sizeof(lf::MulRec) + lf::mem32_bytes(1, (int)std::max<size_t>(1, nb)) +
         sizeof(lf::MemRec64) * std::max<size_t>(1, nb);
}

void* take(lf_server* s, Req& q, size_t bytes) {
  void* p = s->arena.alloc(bytes);
  if (p) q.blocks.push_back({p, bytes});
  return p;
}
void give_back(lf_server* s, Req& q) {
  for (auto& b : q.blocks) s->arena.release(b.first, b.second);
  q.blocks.clear();
}

// Place a chi^2 request's buffers in the arena; false when it does not fit now.
bool admit_chi2(lf_server* s, Req& q) {
  const lf_request& r = q.r;
  size_t S = r.S, n = S * r.cons->n_img;
  lf::Chi2Args& A = q.A;
  std::memset(&A, 0, sizeof A);
  bool ok = true;
  auto get = [&](size_t b) { void* p = ok ? take(s, q, b) : nullptr; if (!p) ok = false; return p; };
  q.d_params = (double*)get(sizeof(double) * std::max<size_t>(1, S * r.model->n_free));
  A.chi2 = (double*)get(sizeof(double) * S);
  A.flags = (int*)get(sizeof(int) * S);
  A.mains = (lf::MainRec*)get(sizeof(lf::MainRec) * std::max<size_t>(1, S * r.model->main.size()));
  A.muls = (lf::MulRec*)get(sizeof(lf::MulRec) * S);
  A.part = (double*)get(sizeof(double) * n * 5);
  A.pflags = (int*)get(sizeof(int) * n);
  A.wimg = (double*)get(sizeof(double) * n * 6);
  A.csrc = (double*)get(sizeof(double) * n);
  A.cimg = (double*)get(sizeof(double) * n);
  A.iflags = (int*)get(sizeof(int) * n);
  A.bm_ws = (double*)get(sizeof(double) * S * r.cons->n_fam * 2);
  A.strag_n = (int*)get(sizeof(int));
  if (!ok) { give_back(s, q); return false; }
  A.n_cu = s->ctx->n_cu > 0 ? s->ctx->n_cu : 256;
  A.m = lf_dev_model(r.model);
  A.cat32 = r.model->d_cat32;
  A.S = r.S; A.n_img = r.cons->n_img; A.n_fam = r.cons->n_fam;
  A.th = r.cons->d_theta; A.fam = r.cons->d_fam; A.fam_start = r.cons->d_fam_start; A.afam = r.cons->d_afam;
  A.sinv = r.cons->d_sinv; A.sigmax = r.cons->d_sigmax;
  A.bmod = nullptr; A.tmod = nullptr;
  A.newton_tol = 1e-9;
  lf::QuadTab qt = lf_quad(s->ctx);
  A.qd.n = qt.n; A.qd.u = qt.u; A.qd.w = qt.w;
  return true;
}

bool admit_map(lf_server* s, Req& q) {
  const lf_request& r = q.r;
  q.P = (long long)r.grid.nx * r.grid.ny;
  q.n_planes = map_planes(r.kind);
  size_t nb = std::max<size_t>(1, r.model->mem.size());
  long long chunkP = (long long)s->cfg.map_chunk_rows * r.grid.nx;
  bool ok = true;
  auto get = [&](size_t b) { void* p = ok ? take(s, q, b) : nullptr; if (!p) ok = false; return p; };
  q.d_params = (double*)get(sizeof(double) * std::max<size_t>(1, r.model->n_free));
  if (r.out_device) {
    // result in the caller's device memory; without flags_device, chunk-sized scratch for the
    // flags every chunk writes
    q.d_out = r.out_device;
    q.d_flags = r.flags_device ? r.flags_device : (int*)get(sizeof(int) * chunkP);
  } else {
    q.d_out = (double*)get(sizeof(double) * q.n_planes * q.P);
    q.d_flags = (int*)get(sizeof(int) * q.P);
  }
  q.part = (double*)get(chunkP * (sizeof(double) * 9 + sizeof(int)));
  q.mains = (lf::MainRec*)get(sizeof(lf::MainRec) * std::max<size_t>(1, r.model->main.size()));
  q.muls = (lf::MulRec*)get(sizeof(lf::MulRec));
  q.m32 = (lf::MemRec32*)get(lf::mem32_bytes(1, (int)nb));
  q.m64 = (lf::MemRec64*)get(sizeof(lf::MemRec64) * nb);
  if (!ok) { give_back(s, q); return false; }
  return true;
}

void finish(lf_server* s, Req& q, int status) {
  q.status = status;
  q.t_done = Clock::now();
  give_back(s, q);
}

// Launch all admitted, not yet launched chi^2 requests of one (mode, precision) as one batch.
void launch_chi2_batch(lf_server* s) {
  std::vector<std::shared_ptr<Req>> todo;
  for (auto& q : s->admitted_chi2)
    if (!q->launched) todo.push_back(q);
  if (todo.empty()) return;
  int mode = todo[0]->r.mode, prec = todo[0]->r.prec;
  std::vector<std::shared_ptr<Req>> batch;
  long long samples = 0;
  for (auto& q : todo)
    if (q->r.mode == mode && q->r.prec == prec && samples + q->r.S <= s->cfg.max_batch_samples) {
      batch.push_back(q);
      samples += q->r.S;
    }
  if (batch.empty()) batch.push_back(todo[0]);
  // keep the batch's tables within the reserved region
  auto table_bytes = [](size_t items, size_t tiles, size_t samples) {
    return ((sizeof(lf::Chi2Args) * items + 255) & ~(size_t)255) + ((sizeof(lf::BatchTile) * tiles + 255) & ~(size_t)255) +
           sizeof(int) * 2 * samples + 256;
  };
  {
    size_t items = 0, tiles = 0, samples = 0;
    size_t keep = 0;
    for (auto& q : batch) {
      size_t t = ((size_t)q->r.S * q->A.n_img + 255) / 256;
      if (keep > 0 && table_bytes(items + 1, tiles + t, samples + q->r.S) > TABLE_BYTES) break;
      items += 1; tiles += t; samples += q->r.S; ++keep;
    }
    batch.resize(keep);
  }
  hipStream_t st = s->streams[0];
  Unit u;
  u.stream = 0;
  std::vector<lf::Chi2Args>& args = u.args;
  std::vector<std::pair<long long, lf::BatchTile>> tiles;
  std::vector<int>& sl = u.samp;
  std::vector<int> samp;
  for (size_t i = 0; i < batch.size(); ++i) {
    Req& q = *batch[i];
    if (q.r.model->n_free > 0)
      hipMemcpyAsync(q.d_params, q.params.data(), sizeof(double) * q.params.size(), hipMemcpyHostToDevice, st);
    lf::launch_expand(q.A.m, q.r.model->n_free > 0 ? q.d_params : nullptr, q.r.S, (lf::MainRec*)q.A.mains,
                      (lf::MulRec*)q.A.muls, nullptr, nullptr, st);
    args.push_back(q.A);
    long long n = (long long)q.r.S * q.A.n_img;
    long long cost = (long long)(q.r.model->main.size() * 8 + q.r.model->mem.size());
    for (long long g0 = 0; g0 < n; g0 += 256) {
      lf::BatchTile T;
      T.item = (int)i; T.pad = 0; T.g0 = g0; T.g1 = std::min(n, g0 + 256);
      tiles.push_back({cost * (T.g1 - T.g0), T});
    }
    for (int k = 0; k < q.r.S; ++k) samp.push_back((int)i);
  }
  std::stable_sort(tiles.begin(), tiles.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<lf::BatchTile>& ht = u.tiles;
  ht.resize(tiles.size());
  for (size_t k = 0; k < tiles.size(); ++k) ht[k] = tiles[k].second;
  int total = (int)samp.size();
  sl.resize(2 * total);
  {
    int k = 0;
    for (size_t i = 0; i < batch.size(); ++i)
      for (int j = 0; j < batch[i]->r.S; ++j) { sl[k] = (int)i; sl[total + k] = j; ++k; }
  }
  size_t b_args = sizeof(lf::Chi2Args) * args.size(), b_tiles = sizeof(lf::BatchTile) * ht.size(),
         b_samp = sizeof(int) * sl.size();
  char* d_args = s->tables;
  char* d_tiles = d_args + ((b_args + 255) & ~(size_t)255);
  char* d_samp = d_tiles + ((b_tiles + 255) & ~(size_t)255);
  char* d_cnt = d_samp + ((b_samp + 255) & ~(size_t)255);
  hipMemcpyAsync(d_args, args.data(), b_args, hipMemcpyHostToDevice, st);
  hipMemcpyAsync(d_tiles, ht.data(), b_tiles, hipMemcpyHostToDevice, st);
  hipMemcpyAsync(d_samp, sl.data(), b_samp, hipMemcpyHostToDevice, st);
  lf::BatchArgs B;
  B.items = (const lf::Chi2Args*)d_args; B.n_items = (int)args.size();
  B.tiles = (const lf::BatchTile*)d_tiles; B.n_tiles = (int)ht.size();
  B.counter = (int*)d_cnt;
  B.samp_item = (const int*)d_samp; B.samp_local = (const int*)d_samp + total; B.total_S = total;
  int n_cu = s->ctx->n_cu > 0 ? s->ctx->n_cu : 256;
  lf::launch_batch(B, prec == LF_PREC_MIXED, mode, 256, n_cu * 4, st);
  for (auto& q : batch) {
    hipMemcpyAsync(q->r.out_host, q->A.chi2, sizeof(double) * q->r.S, hipMemcpyDeviceToHost, st);
    if (q->r.flags_host)
      hipMemcpyAsync(q->r.flags_host, q->A.flags, sizeof(int) * q->r.S, hipMemcpyDeviceToHost, st);
    q->launched = true;
  }
  u.ev = s->ev();
  hipEventRecord(u.ev, st);
  u.reqs = batch;
  s->busy[0] = true;
  s->inflight.push_back(std::move(u));   // moved: the host buffers the copies read stay alive
}

void launch_map_chunk(lf_server* s, int si, const std::shared_ptr<Req>& qp) {
  Req& q = *qp;
  hipStream_t st = s->streams[si];
  const lf_request& r = q.r;
  if (!q.expanded) {
    if (r.model->n_free > 0)
      hipMemcpyAsync(q.d_params, q.params.data(), sizeof(double) * q.params.size(), hipMemcpyHostToDevice, st);
    lf::launch_expand(lf_dev_model(r.model), r.model->n_free > 0 ? q.d_params : nullptr, 1, q.mains, q.muls, q.m32,
                      q.m64, st);
    q.expanded = true;
  }
  int rows = std::min(s->cfg.map_chunk_rows, r.grid.ny - q.next_row);
  long long off = (long long)q.next_row * r.grid.nx;
  lf::PointsSpec ps;
  ps.grid = 1; ps.x0 = r.grid.x0; ps.y0 = r.grid.y0; ps.h = r.grid.h; ps.nx = r.grid.nx; ps.ny = r.grid.ny;
  ps.px = ps.py = nullptr; ps.P = (long long)rows * r.grid.nx; ps.p0 = off;
  lf::MapsOut o;
  std::memset(&o, 0, sizeof o);
  bool d3 = r.kind == LF_REQ_SING_MAP;
  if (d3) {
    o.kappa = q.d_out + off; o.detA = q.d_out + q.P + off; o.e1 = q.d_out + 2 * q.P + off;
    o.e2 = q.d_out + 3 * q.P + off; o.f1 = q.d_out + 4 * q.P + off; o.f2 = q.d_out + 5 * q.P + off;
  } else {
    o.mu = q.d_out + off;
  }
  o.flags = (r.out_device && !r.flags_device) ? q.d_flags : q.d_flags + off;   // (outputs are chunk-relative)
  lf::DevModel dm = lf_dev_model(r.model);
  bool mixed = r.prec == LF_PREC_MIXED;
  double* part = lf::has_heavy(dm) ? q.part : nullptr;
  int ppl = s->ctx->maps_ppl(mixed, d3);
  if (part) lf::launch_maps(dm, q.mains, q.m32, q.m64, 1, ps, r.a_dis, mixed, d3, o, lf_quad(s->ctx), ppl, part, 1, st);
  lf::launch_maps(dm, q.mains, q.m32, q.m64, 1, ps, r.a_dis, mixed, d3, o, lf_quad(s->ctx), ppl, part, 2, st);
  q.next_row += rows;
  const size_t n = (size_t)rows * r.grid.nx;
  if (r.out_host) {
    for (int p = 0; p < q.n_planes; ++p)
      hipMemcpyAsync((double*)r.out_host + p * q.P + off, q.d_out + p * q.P + off, sizeof(double) * n,
                     hipMemcpyDeviceToHost, st);
    if (r.flags_host)
      hipMemcpyAsync((int*)r.flags_host + off, q.d_flags + off, sizeof(int) * n, hipMemcpyDeviceToHost, st);
  }
  Unit u;
  u.stream = si;
  u.last_chunk = q.next_row >= r.grid.ny;
  u.map = qp;
  u.ev = s->ev();
  hipEventRecord(u.ev, st);
  s->busy[si] = true;
  s->inflight.push_back(std::move(u));   // moved: the host buffers the copies read stay alive
}

}  // namespace

void lf_server::loop() {
  hipSetDevice(ctx->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      bool idle = inflight.empty() && incoming.empty() && pending.empty() && admitted_chi2.empty() &&
                  maps_queue.empty();
      if (idle && map_bound.empty()) {
        if (stop) break;
        cv.wait_for(lk, std::chrono::milliseconds(2));
      }
      while (!incoming.empty()) { pending.push_back(incoming.front()); incoming.pop_front(); }
      if (stop) {   // requests not yet admitted fail; admitted work drains
        for (auto& q : pending) { q->status = LF_E_NOT_READY; q->t_done = Clock::now(); }
        pending.clear();
        done_cv.notify_all();
      }
    }
    bool progressed = false;
    // completions
    for (size_t k = 0; k < inflight.size();) {
      Unit& u = inflight[k];
      if (hipEventQuery(u.ev) == hipSuccess) {
        ev_pool.push_back(u.ev);
        busy[u.stream] = false;
        std::lock_guard<std::mutex> lk(mu);
        if (!u.map) {
          for (auto& q : u.reqs) {
            finish(this, *q, 1);
            admitted_chi2.erase(std::find(admitted_chi2.begin(), admitted_chi2.end(), q));
          }
        } else if (u.last_chunk) {
          finish(this, *u.map, 1);
          map_bound.erase(std::find(map_bound.begin(), map_bound.end(), u.map));
        }
        done_cv.notify_all();
        inflight.erase(inflight.begin() + k);
        progressed = true;
      } else {
        ++k;
      }
    }
    // admission in arrival order; a request that cannot fit now does not block later ones
    for (size_t k = 0; k < pending.size();) {
      auto q = pending[k];
      bool ok = q->r.kind == LF_REQ_CHI2 ? admit_chi2(this, *q) : admit_map(this, *q);
      if (ok) {
        q->admitted = true;
        if (q->r.kind == LF_REQ_CHI2) admitted_chi2.push_back(q);
        else maps_queue.push_back(q);
        pending.erase(pending.begin() + k);
        progressed = true;
      } else {
        ++k;
      }
    }
    if (!busy[0]) launch_chi2_batch(this);
    for (int si = 1; si < (int)streams.size(); ++si) {
      if (busy[si]) continue;
      // shortest remaining work among this stream's unfinished maps and the unbound ones
      std::shared_ptr<Req> best;
      for (auto& q : map_bound)
        if (q->stream == si && q->next_row < q->r.grid.ny && (!best || q->remaining() < best->remaining())) best = q;
      for (auto& q : maps_queue)
        if (!best || q->remaining() < best->remaining()) best = q;
      if (!best) continue;
      if (best->stream < 0) {
        best->stream = si;
        maps_queue.erase(std::find(maps_queue.begin(), maps_queue.end(), best));
        map_bound.push_back(best);
      }
      launch_map_chunk(this, si, best);
      progressed = true;
    }
    if (!progressed && !inflight.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

extern "C" lf_status lf_serve_start(lf_ctx* ctx, const lf_serve_config* cfg, lf_server** out) {
  if (!ctx || !cfg || !out) return LF_E_INVALID_ARG;
  *out = nullptr;
  if (cfg->n_streams < 2 || cfg->n_streams > 8 || cfg->hbm_budget < (1u << 20))
    return ctx->fail(LF_E_INVALID_ARG, "serve: need 2..8 streams and a budget >= 1 MiB");
  hipSetDevice(ctx->device);
  lf_server* s = new lf_server();
  s->ctx = ctx;
  s->cfg = *cfg;
  if (s->cfg.max_batch_samples <= 0) s->cfg.max_batch_samples = 65536;
  if (s->cfg.map_chunk_rows <= 0) s->cfg.map_chunk_rows = 256;
  if (ctx->dev_bytes + cfg->hbm_budget + TABLE_BYTES > ctx->budget || !s->arena.init(cfg->hbm_budget) ||
      hipMalloc((void**)&s->tables, TABLE_BYTES) != hipSuccess) {
    if (s->arena.base) hipFree(s->arena.base);
    delete s;
    return ctx->fail(LF_E_OUT_OF_BUDGET, "serve: cannot reserve %zu bytes", cfg->hbm_budget);
  }
  ctx->dev_bytes += cfg->hbm_budget + TABLE_BYTES;
  s->streams.resize(cfg->n_streams);
  for (auto& st : s->streams) hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  s->busy.assign(cfg->n_streams, false);
  s->th = std::thread([s]() { s->loop(); });
  *out = s;
  return LF_OK;
}

extern "C" lf_status lf_serve_submit(lf_server* s, const lf_request* req, int64_t* ticket) {
  if (!s || !req || !ticket) return LF_E_INVALID_ARG;
  const lf_request& r = *req;
  if (!r.model || (r.prec != LF_PREC_FP64 && r.prec != LF_PREC_MIXED)) return LF_E_INVALID_ARG;
  const bool map = r.kind == LF_REQ_MU_MAP || r.kind == LF_REQ_SING_MAP;
  if (map ? (!r.out_host == !r.out_device) : (!r.out_host || r.out_device)) return LF_E_INVALID_ARG;
  auto q = std::make_shared<Req>();
  q->r = r;
  if (r.kind == LF_REQ_CHI2) {
    if (!r.cons || r.S < 1 || (r.mode != 0 && r.mode != 1) || (r.model->n_free > 0 && !r.params)) return LF_E_INVALID_ARG;
    if (r.mode == 1 && (long long)r.S * r.cons->n_img >= (1LL << 31)) return LF_E_INVALID_ARG;
    if (r.cons->has_obs()) return LF_E_UNSUPPORTED;      // flux / delay terms: lf_chi2_terms
    size_t tiles = ((size_t)r.S * r.cons->n_img + 255) / 256;
    if (sizeof(lf::Chi2Args) + sizeof(lf::BatchTile) * tiles + sizeof(int) * 2 * (size_t)r.S + 1024 > TABLE_BYTES)
      return LF_E_OUT_OF_BUDGET;
    if (r.model->n_free > 0) q->params.assign(r.params, r.params + (size_t)r.S * r.model->n_free);
    q->footprint = chi2_footprint(r);
  } else if (r.kind == LF_REQ_MU_MAP || r.kind == LF_REQ_SING_MAP) {
    if (r.grid.nx < 1 || r.grid.ny < 1 || !(r.grid.h > 0) || !(r.a_dis > 0) || (r.model->n_free > 0 && !r.params))
      return LF_E_INVALID_ARG;
    if (r.model->n_free > 0) q->params.assign(r.params, r.params + r.model->n_free);
    q->footprint = map_footprint(s, r);
  } else {
    return LF_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return LF_E_INVALID_ARG;
  q->id = s->next_id++;
  q->t_submit = Clock::now();
  s->all[q->id] = q;
  if (q->footprint + 4096 > s->cfg.hbm_budget) {
    q->status = LF_E_OUT_OF_BUDGET;
    q->t_done = q->t_submit;
  } else {
    s->incoming.push_back(q);
    s->cv.notify_one();
  }
  *ticket = q->id;
  return LF_OK;
}

extern "C" lf_status lf_serve_poll(lf_server* s, int64_t ticket, int32_t* status, double* latency_ms) {
  if (!s || !status) return LF_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return LF_E_INVALID_ARG;
  *status = it->second->status;
  if (latency_ms)
    *latency_ms = it->second->status != 0
                      ? std::chrono::duration<double, std::milli>(it->second->t_done - it->second->t_submit).count()
                      : -1.0;
  return LF_OK;
}

extern "C" lf_status lf_serve_wait(lf_server* s, int64_t ticket, int32_t* status, double* latency_ms) {
  if (!s || !status) return LF_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return LF_E_INVALID_ARG;
  auto q = it->second;
  s->done_cv.wait(lk, [&]() { return q->status != 0; });
  *status = q->status;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
  return LF_OK;
}

extern "C" lf_status lf_serve_stats(lf_server* s, int32_t kind, int64_t* count, double* p50, double* p99,
                                    double* mean) {
  if (!s) return LF_E_INVALID_ARG;
  std::vector<double> v;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& kv : s->all) {
      const Req& q = *kv.second;
      if (q.status == 1 && (kind < 0 || q.r.kind == kind))
        v.push_back(std::chrono::duration<double, std::milli>(q.t_done - q.t_submit).count());
    }
  }
  std::sort(v.begin(), v.end());
  auto pct = [&](double p) {
    if (v.empty()) return 0.0;
    double x = p * (v.size() - 1);
    size_t i = (size_t)x;
    double f = x - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
  };
  if (count) *count = (int64_t)v.size();
  if (p50) *p50 = pct(0.5);
  if (p99) *p99 = pct(0.99);
  if (mean) {
    double m = 0;
    for (double x : v) m += x;
    *mean = v.empty() ? 0.0 : m / v.size();
  }
  return LF_OK;
}

extern "C" lf_status lf_serve_stop(lf_server* s) {
  if (!s) return LF_E_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  s->th.join();
  for (auto st : s->streams) { hipStreamSynchronize(st); hipStreamDestroy(st); }
  for (auto e : s->ev_pool) hipEventDestroy(e);
  hipFree(s->arena.base);
  hipFree(s->tables);
  s->ctx->dev_bytes -= s->cfg.hbm_budget + TABLE_BYTES;
  delete s;
  return LF_OK;
}

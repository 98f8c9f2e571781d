// Uneven batched chi^2: plans, hipGraph capture, tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <vector>

#include "lf_api_internal.h"
#include "lf_chi2.h"

struct lf_batch {
  lf_ctx* ctx = nullptr;
  int mode = 0;
  bool mixed = true;
  std::vector<lf_batch_item> items;
  std::vector<lf::Chi2Args> args;
  std::vector<std::pair<void*, size_t>> allocs;
  lf::Chi2Args* d_args = nullptr;
  lf::BatchTile* d_tiles = nullptr;
  size_t tiles_cap = 0;
  int n_tiles = 0;
  int* d_counter = nullptr;
  int* d_samp = nullptr;
  int total_S = 0;
  int block = 256, grid = 1024, tile_lanes = 256;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<long long> item_cost;   // halos per lane of each item
};

namespace {

lf_status balloc(lf_batch* b, void** p, size_t bytes) {
  lf_status e = b->ctx->dmalloc(p, bytes);
  if (e == LF_OK) b->allocs.push_back({*p, bytes});
  return e;
}

std::string cache_path() {
  const char* e = std::getenv("LF_AUTOTUNE_CACHE");
  if (e && *e) return e;
  const char* h = std::getenv("HOME");
  std::string dir = std::string(h ? h : "/tmp") + "/.cache/lensfield";
  mkdir((std::string(h ? h : "/tmp") + "/.cache").c_str(), 0755);
  mkdir(dir.c_str(), 0755);
  return dir + "/autotune.txt";
}

int ilog2(double x) { return x <= 1 ? 0 : (int)std::floor(std::log2(x)); }

lf_status build_tiles(lf_batch* b, int tile_lanes) {
  std::vector<std::pair<long long, lf::BatchTile>> t;
  for (size_t i = 0; i < b->args.size(); ++i) {
    long long n = (long long)b->args[i].S * b->args[i].n_img;
    for (long long g0 = 0; g0 < n; g0 += tile_lanes) {
      lf::BatchTile T;
      T.item = (int)i; T.pad = 0; T.g0 = g0; T.g1 = std::min(n, g0 + tile_lanes);
      t.push_back({b->item_cost[i] * (T.g1 - T.g0), T});
    }
  }
  std::stable_sort(t.begin(), t.end(), [](const auto& a, const auto& c) { return a.first > c.first; });
  std::vector<lf::BatchTile> h(t.size());
  for (size_t k = 0; k < t.size(); ++k) h[k] = t[k].second;
  if (h.size() > b->tiles_cap) {
    if (b->d_tiles) {
      for (auto it = b->allocs.begin(); it != b->allocs.end(); ++it)
        if (it->first == b->d_tiles) { b->ctx->dfree(it->first, it->second); b->allocs.erase(it); break; }
    }
    lf_status e = balloc(b, (void**)&b->d_tiles, sizeof(lf::BatchTile) * h.size());
    if (e) return e;
    b->tiles_cap = h.size();
  }
  hipMemcpy(b->d_tiles, h.data(), sizeof(lf::BatchTile) * h.size(), hipMemcpyHostToDevice);
  b->n_tiles = (int)h.size();
  b->tile_lanes = tile_lanes;
  return LF_OK;
}

lf::BatchArgs batch_args(const lf_batch* b) {
  lf::BatchArgs B;
  B.items = b->d_args; B.n_items = (int)b->args.size();
  B.tiles = b->d_tiles; B.n_tiles = b->n_tiles;
  B.counter = b->d_counter;
  B.samp_item = b->d_samp; B.samp_local = b->d_samp + b->total_S;
  B.total_S = b->total_S;
  return B;
}

}  // namespace

extern "C" lf_status lf_batch_release(lf_batch* b) {
  if (!b) return LF_E_INVALID_ARG;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->cap_stream) { hipStreamSynchronize(b->cap_stream); hipStreamDestroy(b->cap_stream); }
  for (auto& a : b->allocs) b->ctx->dfree(a.first, a.second);
  delete b;
  return LF_OK;
}

extern "C" lf_status lf_batch_create(lf_ctx* ctx, const lf_batch_item* items, int32_t n_items, int32_t mode,
                                     lf_prec prec, int32_t autotune, lf_batch** out) {
  if (!ctx || !out) return LF_E_INVALID_ARG;
  *out = nullptr;
  if (!items || n_items < 1) return ctx->fail(LF_E_INVALID_ARG, "empty batch");
  if (mode != 0 && mode != 1) return ctx->fail(LF_E_INVALID_ARG, "mode must be 0 or 1");
  if (prec != LF_PREC_FP64 && prec != LF_PREC_MIXED) return ctx->fail(LF_E_INVALID_ARG, "bad precision");
  for (int i = 0; i < n_items; ++i) {
    const lf_batch_item& it = items[i];
    if (!it.model || !it.cons || !it.chi2 || it.S < 1 || (it.model->n_free > 0 && !it.params))
      return ctx->fail(LF_E_INVALID_ARG, "batch item %d: bad model/constraints/samples/output", i);
    if (it.cons->has_obs())
      return ctx->fail(LF_E_UNSUPPORTED, "batch item %d: flux / time-delay constraints are served by lf_chi2_terms", i);
    if (mode == 1 && (long long)it.S * it.cons->n_img >= (1LL << 31))
      return ctx->fail(LF_E_INVALID_ARG, "batch item %d: image plane needs S * n_img < 2^31", i);
  }
  hipSetDevice(ctx->device);
  lf_batch* b = new lf_batch();
  b->ctx = ctx;
  b->mode = mode;
  b->mixed = prec == LF_PREC_MIXED;
  b->items.assign(items, items + n_items);
  hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  lf_status e = LF_OK;
  std::vector<int> samp;
  for (int i = 0; i < n_items; ++i) {
    const lf_batch_item& it = items[i];
    const lf_model* M = it.model;
    const lf_cons* c = it.cons;
    size_t S = it.S, n = S * c->n_img;
    lf::Chi2Args A;
    std::memset(&A, 0, sizeof A);
    lf::MainRec* mains; lf::MulRec* muls;
    e = balloc(b, (void**)&mains, sizeof(lf::MainRec) * std::max<size_t>(1, S * M->main.size())); if (e) break;
    e = balloc(b, (void**)&muls, sizeof(lf::MulRec) * S); if (e) break;
    e = balloc(b, (void**)&A.part, sizeof(double) * n * 5); if (e) break;
    e = balloc(b, (void**)&A.pflags, sizeof(int) * n); if (e) break;
    e = balloc(b, (void**)&A.wimg, sizeof(double) * n * 6); if (e) break;
    e = balloc(b, (void**)&A.csrc, sizeof(double) * n); if (e) break;
    e = balloc(b, (void**)&A.cimg, sizeof(double) * n); if (e) break;
    e = balloc(b, (void**)&A.iflags, sizeof(int) * n); if (e) break;
    e = balloc(b, (void**)&A.bm_ws, sizeof(double) * S * c->n_fam * 2); if (e) break;
    e = balloc(b, (void**)&A.strag_n, sizeof(int)); if (e) break;
    A.n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
    A.m = lf_dev_model(M);
    A.mains = mains; A.muls = muls; A.cat32 = M->d_cat32;
    A.S = it.S; A.n_img = c->n_img; A.n_fam = c->n_fam;
    A.th = c->d_theta; A.fam = c->d_fam; A.fam_start = c->d_fam_start; A.afam = c->d_afam;
    A.sinv = c->d_sinv; A.sigmax = c->d_sigmax;
    A.chi2 = it.chi2; A.flags = it.flags; A.bmod = nullptr; A.tmod = nullptr;
    A.newton_tol = 1e-9;
    lf::QuadTab q = lf_quad(ctx);
    A.qd.n = q.n; A.qd.u = q.u; A.qd.w = q.w;
    b->args.push_back(A);
    b->item_cost.push_back((long long)(M->main.size() * 8 + M->mem.size()));
    for (int s = 0; s < it.S; ++s) samp.push_back(i);
  }
  if (e) { lf_batch_release(b); return e; }
  b->total_S = (int)samp.size();
  std::vector<int> sl(2 * samp.size());
  {
    int k = 0;
    for (int i = 0; i < n_items; ++i)
      for (int s = 0; s < items[i].S; ++s) { sl[k] = i; sl[b->total_S + k] = s; ++k; }
  }
  e = balloc(b, (void**)&b->d_samp, sizeof(int) * sl.size());
  if (!e) e = balloc(b, (void**)&b->d_args, sizeof(lf::Chi2Args) * b->args.size());
  if (!e) e = balloc(b, (void**)&b->d_counter, 64);
  if (e) { lf_batch_release(b); return e; }
  hipMemcpy(b->d_samp, sl.data(), sizeof(int) * sl.size(), hipMemcpyHostToDevice);
  hipMemcpy(b->d_args, b->args.data(), sizeof(lf::Chi2Args) * b->args.size(), hipMemcpyHostToDevice);
  hipStream_t st = b->cap_stream;
  // expansion once, so that autotuning times real halo sums
  for (size_t i = 0; i < b->args.size(); ++i) {
    hipError_t he = lf::launch_expand(b->args[i].m, items[i].params, items[i].S, (lf::MainRec*)b->args[i].mains,
                                      (lf::MulRec*)b->args[i].muls, nullptr, nullptr, st);
    if (he != hipSuccess) { lf_batch_release(b); return ctx->hip(he, "batch expansion"); }
  }
  // default tile shape, or the tuned / cached one
  int n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
  long long lanes = 0, work = 0;
  for (size_t i = 0; i < b->args.size(); ++i) {
    long long n = (long long)b->args[i].S * b->args[i].n_img;
    lanes += n;
    work += n * b->item_cost[i];
  }
  std::ostringstream key;
  key << ctx->arch << "|chi2|m" << mode << "|p" << (b->mixed ? 1 : 0) << "|n" << n_items << "|L" << ilog2((double)lanes)
      << "|W" << ilog2((double)work);
  int best_block = 256, best_tile = 256, best_bpc = 4;
  bool found = false;
  if (autotune) {
    std::ifstream in(cache_path());
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      int bl, tl, bpc;
      if (ls >> k >> bl >> tl >> bpc && k == key.str()) { best_block = bl; best_tile = tl; best_bpc = bpc; found = true; }
    }
    if (!found) {
      hipEvent_t e0, e1;
      hipEventCreate(&e0);
      hipEventCreate(&e1);
      float best = 1e30f;
      const int blocks[3] = {64, 128, 256};
      const int mults[3] = {1, 2, 4};
      const int bpcs[3] = {2, 4, 8};
      for (int bl : blocks)
        for (int mu : mults)
          for (int bpc : bpcs) {
            if ((e = build_tiles(b, bl * mu))) { lf_batch_release(b); return e; }
            lf::BatchArgs B = batch_args(b);
            float tmin = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
              hipEventRecord(e0, st);
              lf::launch_batch_lean_only(B, b->mixed, bl, n_cu * bpc, st);
              hipEventRecord(e1, st);
              hipEventSynchronize(e1);
              float ms = 0;
              hipEventElapsedTime(&ms, e0, e1);
              tmin = std::min(tmin, ms);
            }
            if (tmin < best) { best = tmin; best_block = bl; best_tile = bl * mu; best_bpc = bpc; }
          }
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      std::ofstream o(cache_path(), std::ios::app);
      if (o) o << key.str() << " " << best_block << " " << best_tile << " " << best_bpc << " " << best << "\n";
    }
  }
  b->block = best_block;
  b->grid = n_cu * best_bpc;
  if ((e = build_tiles(b, best_tile))) { lf_batch_release(b); return e; }
  hipStreamSynchronize(st);
  // capture: expansion of every item, counter reset (a kernel), halo sums, reductions
  hipError_t he = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (he == hipSuccess) {
    for (size_t i = 0; i < b->args.size(); ++i)
      lf::launch_expand(b->args[i].m, items[i].params, items[i].S, (lf::MainRec*)b->args[i].mains,
                        (lf::MulRec*)b->args[i].muls, nullptr, nullptr, st);
    lf::launch_batch(batch_args(b), b->mixed, mode, b->block, b->grid, st);
    he = hipStreamEndCapture(st, &b->graph);
  }
  if (he == hipSuccess) he = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (he != hipSuccess) { lf_batch_release(b); return ctx->hip(he, "graph capture"); }
  *out = b;
  return LF_OK;
}

extern "C" lf_status lf_batch_run(lf_batch* b, void* stream) {
  if (!b) return LF_E_INVALID_ARG;
  hipSetDevice(b->ctx->device);
  b->ctx->prof_begin("batch_graph", (hipStream_t)stream);
  hipError_t he = hipGraphLaunch(b->exec, (hipStream_t)stream);
  b->ctx->prof_end((hipStream_t)stream);
  return b->ctx->hip(he, "graph launch");
}

extern "C" lf_status lf_batch_info(const lf_batch* b, int32_t* block, int32_t* grid, int32_t* tile_lanes,
                                   int32_t* n_tiles) {
  if (!b) return LF_E_INVALID_ARG;
  if (block) *block = b->block;
  if (grid) *grid = b->grid;
  if (tile_lanes) *tile_lanes = b->tile_lanes;
  if (n_tiles) *n_tiles = b->n_tiles;
  return LF_OK;
}

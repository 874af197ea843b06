// host_batch.cpp -- host side of batched stepping: the batch handle, its
// tile list and set table, per-set and persistent launches, the hipGraph
// cache and the autotuner.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "host_internal.h"

using namespace soax;
using namespace soax::host;

// Upper bound of blocks_per_cu: with 256 CUs the grid can then cover
// 16.7M tiles, more than the particle limit needs at 128-particle tiles.
constexpr int kMaxBlocksPerCu = 65536;

struct soax_batch {
  std::vector<soax_set*> sets;
  std::vector<uint64_t> generations;  // of each set when the batch was made
  int vel_t = kF32;
  int64_t total = 0;
  // default: one tile per workgroup (the grid covers every tile), one
  // particle per thread -- the fastest shape on the uneven 256-set batch
  int block = 256, per_thread = 1, blocks_per_cu = kMaxBlocksPerCu;
  int cus = 256;
  std::string arch;
  // device tables
  BatchSet* dev_sets = nullptr;
  int32_t* dev_tile_set = nullptr;
  int64_t ntiles = 0;
  int tile_for = 0;  // tile size the tile list was built for
  // host staging of the set table (pinned) and the event guarding its reuse
  BatchSet* stage = nullptr;
  hipEvent_t stage_done = nullptr;
  bool stage_pending = false;
  hipStream_t capture_stream = nullptr;
  std::map<std::tuple<int64_t, int, int, int, int>, hipGraphExec_t> graphs;
  // dt and amplitudes of the most recent step (empty before the first); the
  // tuner times its candidates with them
  std::vector<double> last_dt, last_abc;
  // the largest shift tier among the sets' current dt and amplitudes: the
  // batch kernel is instantiated for tiers up to it
  int max_tier = kTierAny;
};

// --------------------------------------------------------------- batching

namespace {

void drop_graphs(soax_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// (Re)build the tile list for the current tile size and upload it together
// with the set table (whose tile offsets depend on it).  Drains the device
// first: a replaced list may still be read by work in flight.
soax_status build_tiles(soax_batch* b) {
  const int tile = b->block * b->per_thread;
  if (b->tile_for == tile) return SOAX_OK;
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  b->stage_pending = false;
  std::vector<int32_t> tile_set;
  for (size_t si = 0; si < b->sets.size(); ++si) {
    b->stage[si].tile_begin = static_cast<int64_t>(tile_set.size());
    const int64_t nt = (b->sets[si]->n + tile - 1) / tile;
    for (int64_t t = 0; t < nt; ++t) tile_set.push_back(static_cast<int32_t>(si));
  }
  if (tile_set.size() > static_cast<size_t>(INT32_MAX))
    return fail(SOAX_E_RANGE, "too many tiles");
  if (b->dev_tile_set) {
    (void)hipFree(b->dev_tile_set);
    b->dev_tile_set = nullptr;
  }
  b->ntiles = static_cast<int64_t>(tile_set.size());
  if (b->ntiles > 0) {
    hipError_t e = hipMalloc(&b->dev_tile_set, tile_set.size() * sizeof(int32_t));
    if (e != hipSuccess) return fail(SOAX_E_OOM, "hipMalloc(tile list): %s", hipGetErrorString(e));
    HIP_TRY(hipMemcpy(b->dev_tile_set, tile_set.data(), tile_set.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice),
            "hipMemcpy(tile list)");
  }
  HIP_TRY(hipMemcpy(b->dev_sets, b->stage, b->sets.size() * sizeof(BatchSet), hipMemcpyHostToDevice),
          "hipMemcpy(set table)");
  b->tile_for = tile;
  drop_graphs(b);
  return SOAX_OK;
}

BatchLaunch batch_launch(const soax_batch* b) {
  BatchLaunch L{};
  L.sets = b->dev_sets;
  L.tile_set = b->dev_tile_set;
  L.ntiles = b->ntiles;
  L.nsets = static_cast<int32_t>(b->sets.size());
  L.tile = b->block * b->per_thread;
  L.block = b->block;
  L.per_thread = b->per_thread;
  int64_t grid = static_cast<int64_t>(b->cus) * b->blocks_per_cu;
  if (grid > b->ntiles) grid = b->ntiles;
  L.grid = static_cast<int32_t>(std::max<int64_t>(grid, 1));
  L.vel_t = b->vel_t;
  L.max_tier = b->max_tier;
  return L;
}

// Copy dt/abc into the pinned staging table and enqueue its upload.
soax_status upload_params(soax_batch* b, const double* dt, const double* abc, hipStream_t s) {
  if (b->stage_pending) {
    HIP_TRY(hipEventSynchronize(b->stage_done), "hipEventSynchronize");
    b->stage_pending = false;
  }
  b->max_tier = kTierSmall;
  for (size_t i = 0; i < b->sets.size(); ++i) {
    b->stage[i].tier = shift_tier(dt[i], abc[3 * i], abc[3 * i + 1], abc[3 * i + 2]);
    b->max_tier = std::max(b->max_tier, static_cast<int>(b->stage[i].tier));
    b->stage[i].dt = dt[i];
    b->stage[i].A = abc[3 * i];
    b->stage[i].B = abc[3 * i + 1];
    b->stage[i].C = abc[3 * i + 2];
  }
  HIP_TRY(hipMemcpyAsync(b->dev_sets, b->stage, b->sets.size() * sizeof(BatchSet),
                         hipMemcpyHostToDevice, s),
          "hipMemcpyAsync(set table)");
  HIP_TRY(hipEventRecord(b->stage_done, s), "hipEventRecord");
  b->stage_pending = true;
  return SOAX_OK;
}

// A set resized or regrown since the batch was made invalidates the batch's
// tables (sizes, pointers, tiles, captured graphs).
soax_status check_generations(const soax_batch* b) {
  for (size_t i = 0; i < b->sets.size(); ++i)
    if (b->sets[i]->generation != b->generations[i])
      return fail(SOAX_E_STATE, "set %zu changed size since the batch was created", i);
  return SOAX_OK;
}

soax_status per_set_step(soax_batch* b, const double* dt, const double* abc, hipStream_t s) {
  for (size_t i = 0; i < b->sets.size(); ++i) {
    soax_set* set = b->sets[i];
    if (set->n == 0) continue;  // an empty set may have no SoA arrays at all
    const Layout& L = set->L;
    const int fp = L.find("pos"), fv = L.find("vel");
    SoaStepArgs a{};
    for (int d = 0; d < 3; ++d) {
      a.pos[d] = set->soa[L.f[fp].first_array + d];
      a.vel[d] = set->soa[L.f[fv].first_array + d];
    }
    a.n = set->n;
    a.dt = dt[i];
    a.abc = AbcParams{abc[3 * i], abc[3 * i + 1], abc[3 * i + 2]};
    a.wrap = 1;
    // one particle per thread, 128 threads: the faster shape for this mode's
    // mostly cache-resident sets (two per thread in 64 threads took 174 ms
    // against 150 ms for 100 steps of the 256-set batch)
    HIP_TRY(launch_soa_step(kRk2Abc, kF64, b->vel_t, 1, 128, a, s), "per-set step launch");
  }
  return SOAX_OK;
}

soax_status graph_for(soax_batch* b, int64_t nsteps, hipGraphExec_t* out) {
  // the captured kernel handles tiers up to max_tier: a later step whose
  // sets need a larger tier must not replay it
  auto key = std::make_tuple(nsteps, b->block, b->per_thread, b->blocks_per_cu, b->max_tier);
  auto it = b->graphs.find(key);
  if (it != b->graphs.end()) {
    *out = it->second;
    return SOAX_OK;
  }
  const BatchLaunch L = batch_launch(b);
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal),
          "hipStreamBeginCapture");
  hipError_t e = hipSuccess;
  for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) e = launch_batch_rk2(L, b->capture_stream);
  hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(e, "captured batch launch");
  }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  if (b->graphs.size() >= 8) drop_graphs(b);
  b->graphs[key] = ex;
  *out = ex;
  return SOAX_OK;
}

}  // namespace

extern "C" {

soax_status soax_batch_create(soax_set* const* sets, int32_t nsets, soax_batch** out) {
  if (!out) return fail(SOAX_E_ARG, "out is NULL");
  *out = nullptr;
  if (!sets || nsets < 1) return fail(SOAX_E_ARG, "need at least one set");
  int vel_t = 0;
  int64_t total = 0;
  for (int i = 0; i < nsets; ++i) {
    soax_set* s = sets[i];
    if (!s) return fail(SOAX_E_ARG, "sets[%d] is NULL", i);
    int fp, fv;
    soax_status st;
    if ((st = vec_field(s->L, "pos", &fp)) || (st = vec_field(s->L, "vel", &fv))) return st;
    if (s->L.f[fp].dtype != kF64) return fail(SOAX_E_SCHEMA, "batched RK2 needs f64 'pos'");
    if (i == 0) vel_t = s->L.f[fv].dtype;
    if (s->L.f[fv].dtype != vel_t) return fail(SOAX_E_SCHEMA, "every set needs the same 'vel' type");
    if (s->soa.empty() && s->n > 0) return fail(SOAX_E_LAYOUT, "sets[%d] has no SoA copy", i);
    if (s->n > 0 && !s->soa_vec_ok) return fail(SOAX_E_LAYOUT, "sets[%d] arrays are not 16-byte aligned", i);
    total += s->n;
  }
  soax_batch* b = new soax_batch();
  b->sets.assign(sets, sets + nsets);
  for (int i = 0; i < nsets; ++i) b->generations.push_back(sets[i]->generation);
  b->vel_t = vel_t;
  b->total = total;
  int dev = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipGetDeviceProperties");
  }
  b->cus = prop.multiProcessorCount;
  b->arch = prop.gcnArchName;
  soax_status st = SOAX_OK;
  e = hipHostMalloc(reinterpret_cast<void**>(&b->stage), nsets * sizeof(BatchSet), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(&b->dev_sets, nsets * sizeof(BatchSet));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->stage_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) st = hip_fail(e, "batch set-up");
  if (st == SOAX_OK) {
    for (int i = 0; i < nsets; ++i) {
      soax_set* s = sets[i];
      const int fp = s->L.find("pos"), fv = s->L.find("vel");
      BatchSet& t = b->stage[i];
      memset(&t, 0, sizeof t);
      for (int d = 0; d < 3; ++d) {
        t.pos[d] = s->n ? static_cast<double*>(s->soa[s->L.f[fp].first_array + d]) : nullptr;
        t.vel[d] = s->n ? s->soa[s->L.f[fv].first_array + d] : nullptr;
      }
      t.n = s->n;
    }
    st = build_tiles(b);
  }
  if (st != SOAX_OK) {
    soax_batch_destroy(b);
    return st;
  }
  *out = b;
  return SOAX_OK;
}

void soax_batch_destroy(soax_batch* b) {
  if (!b) return;
  if (b->stage_pending) (void)hipEventSynchronize(b->stage_done);
  drop_graphs(b);
  if (b->dev_tile_set) (void)hipFree(b->dev_tile_set);
  if (b->dev_sets) (void)hipFree(b->dev_sets);
  if (b->stage) (void)hipHostFree(b->stage);
  if (b->stage_done) (void)hipEventDestroy(b->stage_done);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  delete b;
}

soax_status soax_batch_config(soax_batch* b, int32_t block, int32_t per_thread, int32_t blocks_per_cu) {
  if (!b) return fail(SOAX_E_ARG, "batch is NULL");
  if (block != 0 && (block < 64 || block > 512 || block % 64))
    return fail(SOAX_E_ARG, "block %d must be 0 or a multiple of 64 in 64..512", block);
  if (per_thread != 0 && per_thread != 1 && per_thread != 2 && per_thread != 4)
    return fail(SOAX_E_ARG, "per_thread %d must be 0, 1, 2 or 4", per_thread);
  if (blocks_per_cu < 0 || blocks_per_cu > kMaxBlocksPerCu)
    return fail(SOAX_E_ARG, "blocks_per_cu must be 0..%d", kMaxBlocksPerCu);
  if (block) b->block = block;
  if (per_thread) b->per_thread = per_thread;
  if (blocks_per_cu) b->blocks_per_cu = blocks_per_cu;
  drop_graphs(b);
  return build_tiles(b);
}

soax_status soax_batch_get_config(const soax_batch* b, int32_t* block, int32_t* per_thread,
                                  int32_t* blocks_per_cu) {
  if (!b) return fail(SOAX_E_ARG, "batch is NULL");
  if (block) *block = b->block;
  if (per_thread) *per_thread = b->per_thread;
  if (blocks_per_cu) *blocks_per_cu = b->blocks_per_cu;
  return SOAX_OK;
}

soax_status soax_batch_step(soax_batch* b, const double* dt, const double* abc, int64_t nsteps,
                            int32_t mode, void* stream) {
  if (!b) return fail(SOAX_E_ARG, "batch is NULL");
  if (!dt || !abc) return fail(SOAX_E_ARG, "dt or abc is NULL");
  if (nsteps < 0) return fail(SOAX_E_ARG, "nsteps is negative");
  if (mode < 0 || mode > 2) return fail(SOAX_E_ARG, "mode must be 0, 1 or 2");
  soax_status st0 = check_generations(b);
  if (st0) return st0;
  for (size_t i = 0; i < b->sets.size(); ++i) {
    if (!is_finite(dt[i])) return fail(SOAX_E_ARG, "dt[%zu] is not finite", i);
    for (int j = 0; j < 3; ++j)
      if (!is_finite(abc[3 * i + j])) return fail(SOAX_E_ARG, "abc[%zu] is not finite", 3 * i + j);
  }
  b->last_dt.assign(dt, dt + b->sets.size());
  b->last_abc.assign(abc, abc + 3 * b->sets.size());
  hipStream_t s = as_stream(stream);
  if (nsteps == 0) return SOAX_OK;
  if (mode == 0) {
    for (int64_t k = 0; k < nsteps; ++k) {
      soax_status st = per_set_step(b, dt, abc, s);
      if (st) return st;
    }
    return SOAX_OK;
  }
  soax_status st = upload_params(b, dt, abc, s);
  if (st) return st;
  if (mode == 1) {
    const BatchLaunch L = batch_launch(b);
    for (int64_t k = 0; k < nsteps; ++k) HIP_TRY(launch_batch_rk2(L, s), "batch launch");
    return SOAX_OK;
  }
  hipGraphExec_t ex = nullptr;
  if ((st = graph_for(b, nsteps, &ex))) return st;
  HIP_TRY(hipGraphLaunch(ex, s), "hipGraphLaunch");
  return SOAX_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tuner

namespace {

struct TuneEntry {
  int block, per_thread, blocks_per_cu;
  double ms;
};

// The cache is a JSON object with one entry per line:
//   "key": {"block": B, "per_thread": P, "blocks_per_cu": C, "ms": T},
std::map<std::string, TuneEntry> read_cache(const char* path) {
  std::map<std::string, TuneEntry> m;
  FILE* f = fopen(path, "r");
  if (!f) return m;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    char key[512];
    TuneEntry e{};
    if (sscanf(line, " \"%511[^\"]\": {\"block\": %d, \"per_thread\": %d, \"blocks_per_cu\": %d, \"ms\": %lf",
               key, &e.block, &e.per_thread, &e.blocks_per_cu, &e.ms) == 5)
      m[key] = e;
  }
  fclose(f);
  return m;
}

bool write_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m) {
    fprintf(f, "\"%s\": {\"block\": %d, \"per_thread\": %d, \"blocks_per_cu\": %d, \"ms\": %.6f}%s\n",
            kv.first.c_str(), kv.second.block, kv.second.per_thread, kv.second.blocks_per_cu,
            kv.second.ms, (++i < m.size()) ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
  return rename(tmp.c_str(), path) == 0;
}

// Device copies of every set's pos and vel, to restore them after timing.
struct Snapshot {
  std::vector<void*> bufs;
  ~Snapshot() {
    for (void* p : bufs) (void)hipFree(p);
  }
};

soax_status snapshot(soax_batch* b, Snapshot& snap, bool restore) {
  size_t k = 0;
  for (soax_set* s : b->sets) {
    if (s->n == 0) continue;
    const int fp = s->L.find("pos"), fv = s->L.find("vel");
    for (int d = 0; d < 3; ++d) {
      for (int which = 0; which < 2; ++which) {
        const Field& f = s->L.f[which ? fv : fp];
        void* arr = s->soa[f.first_array + d];
        const size_t bytes = static_cast<size_t>(s->n) * f.es;
        if (!restore) {
          void* p = nullptr;
          hipError_t e = hipMalloc(&p, bytes);
          if (e != hipSuccess) return fail(SOAX_E_OOM, "hipMalloc(tuning snapshot): %s", hipGetErrorString(e));
          snap.bufs.push_back(p);
          HIP_TRY(hipMemcpy(p, arr, bytes, hipMemcpyDeviceToDevice), "hipMemcpy(snapshot)");
        } else {
          HIP_TRY(hipMemcpy(arr, snap.bufs[k++], bytes, hipMemcpyDeviceToDevice), "hipMemcpy(restore)");
        }
      }
    }
  }
  return SOAX_OK;
}

}  // namespace

extern "C" soax_status soax_batch_tune(soax_batch* b, const char* cache_path) {
  if (!b) return fail(SOAX_E_ARG, "batch is NULL");
  soax_status st0 = check_generations(b);
  if (st0) return st0;
  char keybuf[256];
  snprintf(keybuf, sizeof keybuf, "%s|batch_rk2|vel%d|sets=%zu|n=%lld", b->arch.c_str(), b->vel_t,
           b->sets.size(), static_cast<long long>(b->total));
  const std::string key = keybuf;
  std::map<std::string, TuneEntry> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    auto it = cache.find(key);
    if (it != cache.end())
      return soax_batch_config(b, it->second.block, it->second.per_thread, it->second.blocks_per_cu);
  }
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  Snapshot snap;
  soax_status st = snapshot(b, snap, false);
  if (st) return st;
  // candidates are timed with the most recent step's dt and amplitudes, or
  // dt = 1e-3 and A = B = C = 1 before the first step
  std::vector<double> dts = b->last_dt, abc = b->last_abc;
  if (dts.empty()) {
    dts.assign(b->sets.size(), 1e-3);
    abc.assign(3 * b->sets.size(), 1.0);
  }
  if ((st = upload_params(b, dts.data(), abc.data(), nullptr))) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
  // average time of `reps` launches in one shape, after one warm-up launch
  auto time_shape = [&](const TuneEntry& c, int reps, double* ms_out) -> soax_status {
    soax_status cs = soax_batch_config(b, c.block, c.per_thread, c.blocks_per_cu);
    if (cs) return cs;
    const BatchLaunch L = batch_launch(b);
    hipError_t e = launch_batch_rk2(L, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_batch_rk2(L, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return hip_fail(e, "tuning run");
    *ms_out = ms / reps;
    return SOAX_OK;
  };
  const int blocks[] = {64, 128, 256, 512};
  // four particles per thread splits the 8-byte position runs into
  // half-coalesced 16-byte accesses (measured 2.5x slower): not a candidate
  const int ppts[] = {1, 2};
  // the last candidate gives every tile its own workgroup
  const int bpcs[] = {2, 4, 8, 16, 32, 64, kMaxBlocksPerCu};
  const TuneEntry current{b->block, b->per_thread, b->blocks_per_cu, 0.0};
  // pass 1: every shape, 3 launches each
  std::vector<TuneEntry> timed;
  for (int bl : blocks)
    for (int pp : ppts)
      for (int bc : bpcs) {
        if (st) break;
        TuneEntry c{bl, pp, bc, 0.0};
        if (!(st = time_shape(c, 3, &c.ms))) timed.push_back(c);
      }
  // pass 2: the four fastest and the shape in use, 20 launches each, three
  // times in turn; keep each one's best time (shapes within a few percent of
  // each other swapped places from run to run with two rounds of 10)
  TuneEntry best = current;
  best.ms = 1e30;
  if (!st) {
    std::sort(timed.begin(), timed.end(),
              [](const TuneEntry& x, const TuneEntry& y) { return x.ms < y.ms; });
    std::vector<TuneEntry> finalists(timed.begin(), timed.begin() + std::min<size_t>(4, timed.size()));
    finalists.push_back(current);
    for (TuneEntry& c : finalists) c.ms = 1e30;
    for (int round = 0; round < 3 && !st; ++round)
      for (TuneEntry& c : finalists) {
        double ms = 0.0;
        if ((st = time_shape(c, 20, &ms))) break;
        c.ms = std::min(c.ms, ms);
      }
    for (const TuneEntry& c : finalists)
      if (c.ms < best.ms) best = c;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  soax_status rst = snapshot(b, snap, true);
  if (st) return st;
  if (rst) return rst;
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  if ((st = soax_batch_config(b, best.block, best.per_thread, best.blocks_per_cu))) return st;
  if (cache_path) {
    cache[key] = best;
    if (!write_cache(cache_path, cache)) return fail(SOAX_E_ARG, "cannot write tuning cache '%s'", cache_path);
  }
  return SOAX_OK;
}

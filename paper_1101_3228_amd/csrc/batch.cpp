// Batched forward step + BDP for many contracts with uneven n and N_k:
// per scratch group, two pass-A launches over device work lists of
// (contract, layer, chunk range) units, longest first, one workgroup per
// chunk (one launch for the d >= 2 contracts, one for the 1-D ones), and one
// pass-B launch; then one BDP launch for all (contract, payoff group) pairs,
// captured once into a hipGraph; plus the tuner cache of the launch shapes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "qtree.h"
#include "qtree_batch.hpp"
#include "qtree_plan.hpp"

using qtree::set_error;

struct qtree_tuner {
  std::string path;
  // batch signature -> (configuration code, its measured forward time in ms)
  std::map<std::string, std::pair<int, double>> best;
};

namespace {

// Units [off[x], off[x] + cnt[x]) of a group: x = 0 the 1-D list, x = 1 the
// d >= 2 list; the chunk prefix of list x starts at chunk_base[x] of the
// batch's prefix table and its launch has n_chunks[x] workgroups.
struct Group {
  int unit_off[2] = {0, 0}, n_units[2] = {0, 0}, tile_off = 0, n_tiles = 0;
  int chunk_base[2] = {0, 0}, n_chunks[2] = {0, 0};
};

qtree_status hip_error(hipError_t e, const char* what) {
  return set_error(QTREE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Forced allocation failure, for tests of the error paths: with
// QTREE_FAULT_ALLOC=k (k >= 1) in the environment, the k-th device
// allocation of a call fails as if the device memory were exhausted.
struct AllocFault {
  int fail_at = 0, count = 0;
  AllocFault() {
    const char* v = std::getenv("QTREE_FAULT_ALLOC");
    fail_at = v ? std::atoi(v) : 0;
  }
  hipError_t alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (fail_at > 0 && ++count == fail_at) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
  }
};

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& src, AllocFault& f) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = f.alloc(reinterpret_cast<void**>(dst), sizeof(T) * src.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

// Cache file: one line per batch signature, "qtree-batch <signature> <code> <ms>".
void load_cache(qtree_tuner* t) {
  if (t->path.empty()) return;
  std::ifstream in(t->path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string tag, key;
    int code = 0;
    double ms = 0.0;
    if (ls >> tag >> key >> code >> ms && tag == "qtree-batch") t->best[key] = {code, ms};
  }
}

void save_cache(const qtree_tuner* t) {
  if (t->path.empty()) return;
  std::ofstream out(t->path, std::ios::trunc);
  for (const auto& kv : t->best)
    out << "qtree-batch " << kv.first << " " << kv.second.first << " " << kv.second.second
        << "\n";
}

// Launch configuration of a batch run; counts and values never depend on it.
//   nd_samples: samples per lane sharing each grid read in the d >= 2 launch;
//   overlap:    the 1-D sampling launch runs on a second stream beside the
//               d >= 2 one (both then share the chip), instead of after it;
//   nd_cap:     workgroups per CU of the d >= 2 launch (0: as many as fit),
//               enforced by the launch's dynamic LDS.
struct BatchConfig {
  int nd_samples = 8, overlap = 0, nd_cap = 0;
  int code() const { return (nd_samples == 4 ? 1 : 0) | (overlap << 1) | (nd_cap << 8); }
  static BatchConfig from(int c) {
    BatchConfig k;
    k.nd_samples = (c & 1) ? 4 : 8;
    k.overlap = (c >> 1) & 1;
    k.nd_cap = (c >> 8) & 0xFF;
    return k;
  }
};

}  // namespace

struct qtree_batch {
  int bucketed = 1;  // every 2-D contract's plan has bucket tables in use
  std::vector<qtree_contract> c;
  std::vector<qtree::BatchContract> hc;
  std::vector<qtree::BatchUnit> units;
  std::vector<int32_t> chunk_off;  // per group and list: first chunk of every unit, then the total
  std::vector<qtree::BatchTile> tiles;
  std::vector<qtree::BdpJob> jobs;
  std::vector<qtree::BdpTask> bdp_tasks;  // all backward steps, step by step
  std::vector<int> step_off;              // tasks of step j: [step_off[j], step_off[j + 1])
  int max_last = 0;                       // largest n_pay x N_n of a job
  std::vector<Group> groups;
  std::vector<double> unit_cost;
  qtree::BatchContract* d_contracts = nullptr;
  qtree::BatchUnit* d_units = nullptr;
  int32_t* d_chunk_off = nullptr;
  qtree::BatchTile* d_tiles = nullptr;
  qtree::BdpJob* d_jobs = nullptr;
  qtree::BdpTask* d_bdp_tasks = nullptr;
  uint16_t* d_keys = nullptr;
  uint32_t* d_segs = nullptr;
  int64_t n_v0 = 0;
  size_t lds[2] = {0, 0};     // dynamic LDS of the 1-D and d >= 2 launches
  int dmax = 1;               // largest d among the d >= 2 contracts (1: none)
  int lg1 = 0;                // search depth of the 1-D launch class (log2 of its largest P)
  int gk1 = -1;               // 1-D launch: largest guide K (-1: breadth-first search)
  int sub1 = 1, maxP1 = 1, gtB1 = 1;  // its sub-counters, midpoint slots, largest table
  int subn = 1;                      // sub-counters per tile of the d >= 2 sort
  int cus = 256;
  // workgroups per CU that fit, of each sampling launch: the 1-D one, then the
  // d >= 2 one at 8 and at 4 samples per lane (different kernels)
  int max_per_cu[3] = {1, 1, 1};
  BatchConfig cfg;
  bool cfg_fixed = false;      // set by qtree_batch_set_config: the tuner keeps out
  double tuned_ms = 0.0;       // measured forward time of cfg (0: not measured)
  int candidates = 0;          // configurations timed by the tuner in this process
  qtree_tuner* tuner = nullptr;
  std::string signature;
  bool use_graph = false;
  bool tuned = false;
  hipGraphExec_t exec = nullptr;
  hipStream_t side = nullptr;  // second stream of the overlapped configuration
  hipEvent_t fork = nullptr, join = nullptr;

  ~qtree_batch() {
    if (side) (void)hipStreamSynchronize(side);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
    for (void* p : {(void*)d_contracts, (void*)d_units, (void*)d_chunk_off, (void*)d_tiles,
                    (void*)d_jobs,
                    (void*)d_bdp_tasks,
                    (void*)d_keys, (void*)d_segs})
      if (p) (void)hipFree(p);
  }
};

namespace {

// Arguments of launch x (0: 1-D pass A, 1: d >= 2 pass A) of group g.
qtree::BatchArgs group_args(const qtree_batch* b, const Group& g, int x, const BatchConfig& c) {
  qtree::BatchArgs a{};
  a.contracts = b->d_contracts;
  a.units = b->d_units + g.unit_off[x];
  a.chunk_off = b->d_chunk_off + g.chunk_base[x];
  a.tiles = b->d_tiles + g.tile_off;
  a.n_units = g.n_units[x];
  a.gk = x == 0 ? b->gk1 : -1;
  a.sub = x == 0 ? b->sub1 : b->subn;
  a.maxP = b->maxP1;
  a.gt_Bmax = b->gtB1;
  a.n_tiles = g.n_tiles;
  a.nd_samples = c.nd_samples;
  a.bucketed = (b->dmax == 2 && b->bucketed) ? 1 : 0;
  a.keys = b->d_keys;
  a.segs = b->d_segs;
  return a;
}

// Dynamic LDS of the d >= 2 launch under a configuration: enough for the
// kernel, and with a cap, enough that no more than nd_cap workgroups fit on
// a CU (160 KiB of LDS each).
size_t nd_lds(const qtree_batch* b, const BatchConfig& c) {
  size_t lds = b->lds[1];
  if (c.nd_cap > 0) lds = std::max(lds, (size_t)(160 * 1024) / (size_t)(c.nd_cap + 1) + 16);
  return lds;
}

int nd_fit(const qtree_batch* b, int nd_samples) {
  return b->max_per_cu[nd_samples == 4 ? 2 : 1];
}

int nd_per_cu(const qtree_batch* b, const BatchConfig& c) {
  const int fit = nd_fit(b, c.nd_samples);
  return c.nd_cap > 0 ? std::min(c.nd_cap, fit) : fit;
}

hipError_t ensure_side(qtree_batch* b) {
  hipError_t e = hipSuccess;
  if (!b->side) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
  if (e == hipSuccess && !b->fork) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess && !b->join) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
  return e;
}

// The sampling and histogram launches of every scratch group.
hipError_t enqueue_forward(const qtree_batch* b, const BatchConfig& c, hipStream_t s) {
  for (const Group& g : b->groups) {
    hipError_t e = hipSuccess;
    const bool both = g.n_units[0] > 0 && g.n_units[1] > 0;
    if (c.overlap && both) {
      // the 1-D list on the side stream, the d >= 2 list on s, then join
      e = hipEventRecord(b->fork, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->fork, 0);
      if (e == hipSuccess)
        e = qtree::launch_batch_keys(group_args(b, g, 0, c), 1, b->lg1, g.n_chunks[0], b->lds[0],
                                     b->side);
      if (e == hipSuccess) e = hipEventRecord(b->join, b->side);
      if (e == hipSuccess)
        e = qtree::launch_batch_keys(group_args(b, g, 1, c), b->dmax, b->lg1, g.n_chunks[1],
                                     nd_lds(b, c), s);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join, 0);
    } else {
      for (int x = 1; x >= 0 && e == hipSuccess; --x)  // the heavier d >= 2 list first
        e = qtree::launch_batch_keys(group_args(b, g, x, c), x == 0 ? 1 : b->dmax, b->lg1,
                                     g.n_chunks[x], x == 0 ? b->lds[0] : nd_lds(b, c), s);
    }
    if (e == hipSuccess) e = qtree::launch_batch_count(group_args(b, g, 0, c), s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_all(const qtree_batch* b, hipStream_t s) {
  hipError_t e = enqueue_forward(b, b->cfg, s);
  if (e != hipSuccess) return e;
  return qtree::launch_bdp_steps(b->d_jobs, (int)b->jobs.size(), b->max_last, b->d_bdp_tasks,
                                 b->step_off.data(), (int)b->step_off.size() - 1, s);
}

// The candidate configurations of a batch: samples per lane 8 / 4, serial or
// overlapped sampling launches (when the batch has both kinds), and the d >= 2
// launch at its occupancy limit or one workgroup per CU below it.
std::vector<BatchConfig> candidates(const qtree_batch* b) {
  bool both = false, nd = false;
  for (const Group& g : b->groups) {
    both = both || (g.n_units[0] > 0 && g.n_units[1] > 0);
    nd = nd || g.n_units[1] > 0;
  }
  std::vector<BatchConfig> out;
  for (int ns : {8, 4})
    for (int ov = 0; ov <= (both ? 1 : 0); ++ov)
      for (int cap = 0; cap <= 1; ++cap) {
        BatchConfig c;
        c.nd_samples = ns;
        c.overlap = ov;
        c.nd_cap = cap && nd_fit(b, ns) > 1 ? nd_fit(b, ns) - 1 : 0;
        if (cap && c.nd_cap == 0) continue;
        if (!nd && (ns != 8 || cap)) continue;  // no d >= 2 launch: nothing to vary there
        out.push_back(c);
      }
  return out;
}

// Tuner: a cached configuration for this batch's signature, else every
// candidate's forward launches timed with HIP events on `s` (after one
// warm-up of the first), the fastest kept and written to the cache.
qtree_status tune(qtree_batch* b, hipStream_t s) {
  auto it = b->tuner->best.find(b->signature);
  if (it != b->tuner->best.end()) {
    b->cfg = BatchConfig::from(it->second.first);
    b->tuned_ms = it->second.second;
    return QTREE_OK;
  }
  const std::vector<BatchConfig> cand = candidates(b);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess && cand.size() > 1) e = ensure_side(b);
  if (e == hipSuccess) e = enqueue_forward(b, cand[0], s);  // warm-up
  double best_ms = 0.0;
  BatchConfig best = cand[0];
  for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
    e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = enqueue_forward(b, cand[i], s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (i == 0 || ms < best_ms)) {
      best_ms = ms;
      best = cand[i];
    }
    ++b->candidates;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_error(e, "batch tuning");
  b->cfg = best;
  b->tuned_ms = best_ms;
  b->tuner->best[b->signature] = {best.code(), best_ms};
  save_cache(b->tuner);
  return QTREE_OK;
}

}  // namespace

extern "C" {

qtree_status qtree_tuner_create(const char* cache_path, qtree_tuner** out) {
  if (!out) return set_error(QTREE_EINVAL, "out is NULL");
  qtree_tuner* t = new qtree_tuner;
  if (cache_path) t->path = cache_path;
  else if (const char* env = std::getenv("QTREE_TUNE_CACHE")) t->path = env;
  load_cache(t);
  *out = t;
  return QTREE_OK;
}

void qtree_tuner_destroy(qtree_tuner* t) { delete t; }

int32_t qtree_tuner_lookup(const qtree_tuner* t, const char* signature) {
  if (!t || !signature) return -1;
  auto it = t->best.find(signature);
  return it == t->best.end() ? -1 : it->second.first;
}

qtree_status qtree_batch_plan(const qtree_contract* contracts, int32_t n, qtree_tuner* tuner,
                              size_t scratch_bytes, uint32_t flags, qtree_batch** out) {
  if (!out) return set_error(QTREE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!contracts || n < 1) return set_error(QTREE_EINVAL, "need at least one contract");
  if (scratch_bytes == 0) scratch_bytes = (size_t)4 << 30;
  qtree_batch* b = new qtree_batch;
  b->c.assign(contracts, contracts + n);
  b->tuner = tuner;
  b->use_graph = (flags & 1u) != 0;
  uint64_t sig = 1469598103934665603ull;  // FNV-1a over the batch shape
  auto mix = [&sig](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      sig ^= (v >> (8 * i)) & 0xFF;
      sig *= 1099511628211ull;
    }
  };
  std::vector<int> job_contract;  // contract of every BDP job
  int maxP = 1, maxN = 1, max_tiles1 = 0, max_tilesn = 0;
  int gk = 0, gtB = 1;  // guide tables of the 1-D contracts: largest K (-1 if one has none)
  int64_t v0_off = 0;
  for (int i = 0; i < n; ++i) {
    const qtree_contract& C = contracts[i];
    const qtree_plan* p = C.plan;
    if (!p || !C.counts || !C.phi || !C.V) {
      delete b;
      return set_error(QTREE_EINVAL, "contract " + std::to_string(i) + ": NULL plan or buffer");
    }
    if (C.M < 1 || C.M >= (1ull << 31)) {
      delete b;
      return set_error(QTREE_EOVERFLOW, "contract " + std::to_string(i) + ": M out of range");
    }
    if (C.n_pay < 1) {
      delete b;
      return set_error(QTREE_EINVAL, "contract " + std::to_string(i) + ": n_pay < 1");
    }
    if (!qtree::two_pass_fits(p->d, p->n, p->N.data())) {
      delete b;
      return set_error(QTREE_EUNSUPPORTED,
                       "contract " + std::to_string(i) + ": count blocks too large for batching");
    }
    mix((uint64_t)p->d);
    mix((uint64_t)p->n);
    mix(C.M);
    for (int k = 0; k <= p->n; ++k) mix((uint64_t)p->N[k]);
    b->dmax = std::max(b->dmax, (int)p->d);
    if (p->d == 1) {
      maxP = std::max(maxP, p->maxP);
      max_tiles1 = std::max(max_tiles1, p->max_tiles);
      gk = (gk < 0 || p->gt_Kmax < 0) ? -1 : std::max(gk, (int)p->gt_Kmax);
      gtB = std::max(gtB, (int)p->gt_Bmax);
    } else {
      maxN = std::max(maxN, p->maxN);
      max_tilesn = std::max(max_tilesn, p->max_tiles);
    }
    qtree::BatchContract bc{};
    bc.layers = reinterpret_cast<const qtree::LayerDev*>(p->ws + p->lay.layers);
    bc.mids = reinterpret_cast<const float*>(p->ws + p->lay.aux);
    bc.guide = reinterpret_cast<const uint16_t*>(p->ws + p->lay.guide);
    bc.pts = reinterpret_cast<const float4*>(p->ws + p->lay.points);
    bc.counts = C.counts;
    bc.key0 = (uint32_t)(C.seed & 0xFFFFFFFFu);
    bc.key1 = (uint32_t)(C.seed >> 32);
    bc.contract = C.contract_id;
    bc.d = p->d;
    bc.n = p->n;
    bc.M = C.M;
    bc.chunks = p->d == 1 ? (int32_t)(((C.M + 1) / 2 + qtree::kChunk / 2 - 1) / (qtree::kChunk / 2))
                          : (int32_t)((C.M + qtree::kChunk - 1) / qtree::kChunk);
    bc.seg_stride = p->max_tiles + 1;
    bc.bk_rows = reinterpret_cast<const uint4*>(p->ws + p->lay.bk_rows);
    // the d = 2 launch searches through bucket tables when every 2-D
    // contract has them (results are the same either way)
    if (p->d == 2 && !(p->buckets > 0 && p->tune_buckets)) b->bucketed = 0;
    b->hc.push_back(bc);
    for (int q0 = 0; q0 < C.n_pay; q0 += 16) {
      qtree::BdpJob j{};
      j.layers = bc.layers;
      j.counts = C.counts;
      j.phi = C.phi;
      j.V = C.V;
      j.P = p->points;
      j.n = p->n;
      j.q0 = q0;
      j.nq = std::min(16, C.n_pay - q0);
      b->jobs.push_back(j);
      job_contract.push_back(i);
      b->max_last = std::max(b->max_last, j.nq * p->N[p->n]);
    }
    v0_off += C.n_pay;
  }
  b->n_v0 = v0_off;
  char sbuf[32];
  std::snprintf(sbuf, sizeof(sbuf), "%016llx", (unsigned long long)sig);
  b->signature = sbuf;
  while ((1 << b->lg1) < maxP) ++b->lg1;
  b->lds[0] = qtree::keys_lds_1d(maxP, max_tiles1);
  if (gk >= 0 && qtree::keys_lds_1d_guide(maxP, gtB, max_tiles1) <= 160 * 1024) {
    b->gk1 = gk;
    b->sub1 = qtree::guide_sub_counters(max_tiles1);
    b->maxP1 = maxP;
    b->gtB1 = gtB;
    b->lds[0] = qtree::keys_lds_1d_guide(maxP, gtB, max_tiles1);
  }
  // every d >= 2 contract a bucketed d = 2 one: the launch stages pairs only
  b->lds[1] = (b->dmax == 2 && b->bucketed) ? qtree::keys_lds_nd_bk(maxN, max_tilesn)
                                            : qtree::keys_lds_nd(maxN, max_tilesn);
  b->subn = qtree::nd_sub_counters(max_tilesn);
  if (b->lds[0] > 160 * 1024 || (b->dmax > 1 && b->lds[1] > 160 * 1024)) {
    delete b;
    return set_error(QTREE_EUNSUPPORTED, "batch needs more LDS than a workgroup has");
  }
  for (int x = 0; x < 3; ++x) {
    if (x >= 1 && b->dmax == 1) continue;
    const int lx = x == 0 ? 0 : 1;
    b->max_per_cu[x] =
        std::min(8, qtree::batch_keys_occupancy(x == 0 ? 1 : b->dmax, b->lg1,
                                                x == 0 ? b->gk1 : -1, b->lds[lx], x == 2 ? 4 : 8,
                                                (b->dmax == 2 && b->bucketed) ? 1 : 0));
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    b->cus = prop.multiProcessorCount;

  // scratch groups, then units (longest first within a group) and tiles
  int64_t group_keys = 0, group_segs = 0;
  const size_t per_chunk_key = sizeof(uint16_t) * qtree::kChunk;
  std::vector<int> group_of(n);
  int gi = 0;
  for (int i = 0; i < n; ++i) {
    qtree::BatchContract& bc = b->hc[i];
    const int64_t nk = (int64_t)bc.n * bc.chunks;
    const size_t need = (size_t)nk * per_chunk_key + (size_t)nk * bc.seg_stride * 4;
    if (need > scratch_bytes) {
      delete b;
      return set_error(QTREE_ENOMEM, "contract " + std::to_string(i) +
                                         " alone exceeds the batch scratch");
    }
    const size_t used = (size_t)group_keys * per_chunk_key + (size_t)group_segs * 4;
    if (i > 0 && used + need > scratch_bytes) {
      ++gi;
      group_keys = 0;
      group_segs = 0;
    }
    bc.chunk_base = group_keys;
    bc.seg_base = group_segs;
    group_keys += nk;
    group_segs += nk * bc.seg_stride;
    group_of[i] = gi;
  }
  size_t scratch_keys = 0, scratch_segs = 0;
  {
    // size of the largest group
    std::vector<int64_t> gk(gi + 1, 0), gs(gi + 1, 0);
    for (int i = 0; i < n; ++i) {
      const qtree::BatchContract& bc = b->hc[i];
      gk[group_of[i]] = std::max<int64_t>(gk[group_of[i]], bc.chunk_base + (int64_t)bc.n * bc.chunks);
      gs[group_of[i]] = std::max<int64_t>(gs[group_of[i]],
                                          bc.seg_base + (int64_t)bc.n * bc.chunks * bc.seg_stride);
    }
    for (int x = 0; x <= gi; ++x) {
      scratch_keys = std::max(scratch_keys, (size_t)gk[x]);
      scratch_segs = std::max(scratch_segs, (size_t)gs[x]);
    }
  }
  for (int x = 0; x <= gi; ++x) {
    // cost model: lane-slots per sample (1-D ~200; d >= 2 ~5 per grid point
    // scanned, ~500 in all with the bucket tables)
    std::vector<qtree::BatchUnit> gu;
    std::vector<double> gc;
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
      if (group_of[i] != x) continue;
      const qtree_plan* p = contracts[i].plan;
      for (int k = 0; k < p->n; ++k) {
        const double per =
            p->d == 1 ? 200.0
            : (p->d == 2 && b->bucketed) ? 500.0
                                        : 300.0 + 5.0 * p->d / 2.0 * (p->N[k] + p->N[k + 1]);
        total += per * (double)contracts[i].M;
      }
    }
    const double target = total / (8.0 * 2 * b->cus);  // ~8 units per workgroup slot
    Group grp;
    for (int cls = 0; cls < 2; ++cls) {
      gu.clear();
      gc.clear();
      for (int i = 0; i < n; ++i) {
        const qtree_plan* p = contracts[i].plan;
        if (group_of[i] != x || (p->d > 1) != (cls == 1)) continue;
        const qtree::BatchContract& bc = b->hc[i];
        for (int k = 0; k < p->n; ++k) {
          const double per =
              p->d == 1 ? 200.0 : 300.0 + 5.0 * p->d / 2.0 * (p->N[k] + p->N[k + 1]);
          const double chunk_cost = per * qtree::kChunk;
          int step = (int)std::max(1.0, std::floor(target / chunk_cost));
          step = std::min(step, bc.chunks);
          for (int c0 = 0; c0 < bc.chunks; c0 += step) {
            const int nc = std::min(step, bc.chunks - c0);
            gu.push_back(qtree::BatchUnit{i, k, c0, nc});
            gc.push_back(chunk_cost * nc);
          }
        }
      }
      std::vector<size_t> order(gu.size());
      for (size_t u = 0; u < order.size(); ++u) order[u] = u;
      std::stable_sort(order.begin(), order.end(),
                       [&](size_t a2, size_t b2) { return gc[a2] > gc[b2]; });
      grp.unit_off[cls] = (int)b->units.size();
      grp.n_units[cls] = (int)gu.size();
      grp.chunk_base[cls] = (int)b->chunk_off.size();
      int32_t run = 0;
      for (size_t u : order) {
        b->units.push_back(gu[u]);
        b->unit_cost.push_back(gc[u]);
        b->chunk_off.push_back(run);
        run += gu[u].nchunks;
      }
      b->chunk_off.push_back(run);
      grp.n_chunks[cls] = run;
    }
    grp.tile_off = (int)b->tiles.size();
    for (int i = 0; i < n; ++i) {
      if (group_of[i] != x) continue;
      const qtree_plan* p = contracts[i].plan;
      for (int k = 0; k < p->n; ++k) {
        const int64_t entries = (int64_t)p->N[k] * p->N[k + 1];
        const int st = (int)((entries + qtree::kSuper - 1) / qtree::kSuper);
        for (int t = 0; t < st; ++t) b->tiles.push_back(qtree::BatchTile{i, k, t, 0});
      }
    }
    grp.n_tiles = (int)b->tiles.size() - grp.tile_off;
    b->groups.push_back(grp);
  }

  // backward steps: step j is layer n - 1 - j of every job with n > j
  int max_n = 0;
  for (const qtree::BdpJob& j : b->jobs) max_n = std::max(max_n, (int)j.n);
  b->step_off.assign(1, 0);
  for (int step = 0; step < max_n; ++step) {
    for (size_t jb = 0; jb < b->jobs.size(); ++jb) {
      const qtree::BdpJob& J = b->jobs[jb];
      if (J.n <= step) continue;
      const int k = J.n - 1 - step;
      const int rows = contracts[job_contract[jb]].plan->N[k];
      for (int r0 = 0; r0 < rows; r0 += qtree::kBdpTaskRows)
        b->bdp_tasks.push_back(qtree::BdpTask{(int32_t)jb, k, r0,
                                              std::min(qtree::kBdpTaskRows, rows - r0)});
    }
    b->step_off.push_back((int)b->bdp_tasks.size());
  }
  AllocFault fault;
  hipError_t e = upload(&b->d_contracts, b->hc, fault);
  if (e == hipSuccess) e = upload(&b->d_units, b->units, fault);
  if (e == hipSuccess) e = upload(&b->d_tiles, b->tiles, fault);
  if (e == hipSuccess) e = upload(&b->d_jobs, b->jobs, fault);
  if (e == hipSuccess) e = upload(&b->d_bdp_tasks, b->bdp_tasks, fault);
  if (e == hipSuccess) e = upload(&b->d_chunk_off, b->chunk_off, fault);
  if (e == hipSuccess)
    e = fault.alloc(reinterpret_cast<void**>(&b->d_keys), scratch_keys * per_chunk_key + 16);
  if (e == hipSuccess)
    e = fault.alloc(reinterpret_cast<void**>(&b->d_segs), scratch_segs * sizeof(uint32_t) + 16);
  if (e != hipSuccess) {
    delete b;  // frees what was allocated
    if (e == hipErrorOutOfMemory)
      return set_error(QTREE_ENOMEM, std::string("batch tables: ") + hipGetErrorString(e));
    return hip_error(e, "batch tables");
  }
  *out = b;
  return QTREE_OK;
}

qtree_status qtree_batch_run(qtree_batch* b, double* V0_host, void* stream) {
  if (!b) return set_error(QTREE_EINVAL, "batch is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->tuner && !b->tuned && !b->cfg_fixed) {
    qtree_status st = tune(b, s);
    if (st != QTREE_OK) return st;
    b->tuned = true;
  }
  hipError_t e;
  if (b->cfg.overlap) {
    e = ensure_side(b);
    if (e != hipSuccess) return hip_error(e, "batch side stream");
  }
  if (b->exec) {
    e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hip_error(e, "graph launch");
  } else {
    e = enqueue_all(b, s);
    if (e != hipSuccess) return hip_error(e, "batch launch");
    if (b->use_graph && s != nullptr) {
      // capture the same sequence for the next runs (capture does not execute)
      hipGraph_t graph = nullptr;
      e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e2 = enqueue_all(b, s);
        e = hipStreamEndCapture(s, &graph);
        if (e2 != hipSuccess) e = e2;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_error(e, "graph capture");
    }
  }
  if (V0_host) {
    int64_t at = 0;
    for (const qtree_contract& C : b->c) {
      e = hipMemcpy2DAsync(V0_host + at, sizeof(double), C.V,
                           sizeof(double) * (size_t)C.plan->points, sizeof(double),
                           (size_t)C.n_pay, hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return hip_error(e, "V0 copy");
      at += C.n_pay;
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "stream synchronize");
  }
  return QTREE_OK;
}

qtree_status qtree_batch_info(const qtree_batch* b, int64_t* units, int64_t* tiles,
                              int32_t* groups, int32_t* per_cu_1d, int32_t* per_cu_nd) {
  if (!b) return set_error(QTREE_EINVAL, "batch is NULL");
  if (units) *units = (int64_t)b->units.size();
  if (tiles) *tiles = (int64_t)b->tiles.size();
  if (groups) *groups = (int32_t)b->groups.size();
  if (per_cu_1d) *per_cu_1d = b->max_per_cu[0];
  if (per_cu_nd) *per_cu_nd = nd_per_cu(b, b->cfg);
  return QTREE_OK;
}

qtree_status qtree_batch_tuning(const qtree_batch* b, int32_t* config, double* ms,
                                int32_t* timed) {
  if (!b) return set_error(QTREE_EINVAL, "batch is NULL");
  if (config) *config = b->cfg.code();
  if (ms) *ms = b->tuned_ms;
  if (timed) *timed = b->candidates;
  return QTREE_OK;
}

qtree_status qtree_batch_set_config(qtree_batch* b, int32_t config) {
  if (!b) return set_error(QTREE_EINVAL, "batch is NULL");
  const BatchConfig c = BatchConfig::from(config);
  if (config < 0 || c.code() != config)
    return set_error(QTREE_EINVAL, "unknown configuration code");
  if (c.nd_cap > 8) return set_error(QTREE_EINVAL, "workgroups per CU must be <= 8");
  if (c.nd_cap > 0 && nd_lds(b, c) > 160 * 1024)
    return set_error(QTREE_EINVAL, "workgroup cap below what the kernel's LDS allows");
  if (b->exec) {  // the captured graph holds the old launches
    hipError_t e = hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    if (e != hipSuccess) return hip_error(e, "graph destroy");
  }
  b->cfg = c;
  b->cfg_fixed = true;
  b->tuned_ms = 0.0;
  return QTREE_OK;
}

const char* qtree_batch_signature(const qtree_batch* b) { return b ? b->signature.c_str() : ""; }

void qtree_batch_destroy(qtree_batch* b) { delete b; }

}  // extern "C"

// Device tables of a batch of contracts (many plans in one launch).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qtree_internal.hpp"

namespace qtree {

// One contract: its plan tables, its counts and where its pass-A keys live
// in the batch scratch of its group.
struct BatchContract {
  const LayerDev* layers;
  const float* mids;
  const uint16_t* guide;  // d = 1: the plan's guide tables
  const float4* pts;
  int32_t* counts;
  uint32_t key0, key1, contract;
  int32_t d, n;
  uint64_t M;            // samples per layer, from sample 0
  int64_t chunk_base;    // first chunk slot of layer 0 in the group scratch
  int64_t seg_base;      // first segment word of layer 0 in the group scratch
  int32_t chunks;        // chunks per layer
  int32_t seg_stride;    // tiles of the contract's largest count block + 1
  const uint4* bk_rows;  // d = 2: the plan's bucket rows
};

// Pass-A work unit: chunks [chunk0, chunk0 + nchunks) of layer k of contract c.
struct BatchUnit {
  int32_t c, k, chunk0, nchunks;
};

// Pass-B job: super tile t of layer k of contract c.
struct BatchTile {
  int32_t c, k, t, pad_;
};

struct BatchArgs {
  const BatchContract* contracts;
  const BatchUnit* units;  // this group's units (longest first)
  const int32_t* chunk_off;  // first chunk of every unit in this launch (n_units + 1 entries)
  const BatchTile* tiles;  // this group's tiles
  int32_t n_units, n_tiles;
  // 1-D launch with guide tables (every 1-D contract has them): gk = the
  // batch's largest K (-1: breadth-first search), over maxP midpoints and
  // tables of up to gt_Bmax entries; sub: sub-counters per tile in the sort
  // (of the 1-D or of the d >= 2 launch)
  int32_t gk, sub, maxP, gt_Bmax;
  int32_t nd_samples;  // d >= 2 launch: samples per lane sharing each grid read (8 or 4)
  int32_t bucketed;    // d = 2 launch (every d >= 2 contract 2-D with bucket tables)
  uint16_t* keys;
  uint32_t* segs;
};

// Pass A over a.units, one workgroup per chunk (`grid` = a.chunk_off[n_units]
// chunks): dmax 1 runs the 1-D kernel (every unit must be 1-D), 2 or 3 the
// d >= 2 kernel.
hipError_t launch_batch_keys(const BatchArgs& a, int dmax, int lg1, int grid, size_t lds,
                             hipStream_t s);
// Pass B over a.tiles.
hipError_t launch_batch_count(const BatchArgs& a, hipStream_t s);
// Workgroups of the pass-A kernel (dmax as above; gk >= 0: the 1-D guide
// kernel) that fit on one CU with `lds` bytes of dynamic LDS each.
int batch_keys_occupancy(int dmax, int lg1, int gk, size_t lds, int nd_samples, int bucketed);
size_t keys_lds_1d(int maxP, int max_tiles);
size_t keys_lds_1d_guide(int maxP, int maxB, int max_tiles);
int guide_sub_counters(int max_tiles);
int nd_sub_counters(int max_tiles);
size_t keys_lds_nd(int maxN, int max_tiles);
size_t keys_lds_nd_bk(int maxN, int max_tiles);  // the bucketed d = 2 launches

// BDP of one contract for payoffs [q0, q0 + nq) (nq <= 16).
struct BdpJob {
  const LayerDev* layers;
  const int32_t* counts;
  const double* phi;
  double* V;
  int64_t P;
  int32_t n, q0, nq, pad_;
};

// Rows [row0, row0 + nrows) of layer k of job `job` (nrows <= kBdpTaskRows).
struct BdpTask {
  int32_t job, k, row0, nrows;
};
constexpr int kBdpTaskRows = 16;

// Backward steps of a batch: V_n = phi_n for every job (grid over jobs),
// then step j = 0, 1, ... runs tasks [step_off[j], step_off[j + 1]) -- layer
// n - 1 - j of every job with n > j -- one launch per step.
hipError_t launch_bdp_steps(const BdpJob* jobs, int n_jobs, int max_last, const BdpTask* tasks,
                            const int* step_off, int n_steps, hipStream_t s);

}  // namespace qtree

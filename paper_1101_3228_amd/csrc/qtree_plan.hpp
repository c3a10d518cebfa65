// Host-side plan object shared by the C-ABI implementation files.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "qtree.h"
#include "qtree_internal.hpp"

struct qtree_plan {
  int d = 0, n = 0;
  std::vector<int32_t> N;
  std::vector<int64_t> pt_off, cnt_off, aux_off;
  std::vector<int32_t> P;
  int64_t points = 0, entries = 0, mids_total = 0;
  int32_t maxN = 0, maxP = 0;
  char* ws = nullptr;
  qtree::WsLayout lay{};
  int64_t tune_chunk = 0;  // 0: automatic
  int32_t tune_xcd_map = 1;
  int32_t tune_count = 0;  // 0 automatic, 1 direct atomics, 2 two-pass
  int32_t tune_groups = 0;  // layer groups of the two-pass forward (0: automatic)
  int32_t tune_nd_samples = 8;  // d >= 2 pass A: samples per lane sharing each grid read
  int32_t tune_tail = 100;      // last layer group's share, percent of the others
  int32_t tune_buckets = 1;     // d = 2: cells through the bucket tables
  int64_t buckets = 0;          // d = 2: buckets over all layers (0: no tables)
  int32_t max_tiles = 0, total_tiles = 0;
  std::vector<int32_t> tile_off;  // first super tile of every layer (host copy)
  std::vector<int32_t> unit_off;  // first histogram unit of every layer (host copy)
  std::vector<int32_t> split;     // histogram parts per super tile of every layer
  std::vector<float> marg_L;      // d = 1: the marginal factor L_k of every layer
  std::vector<double> edges;      // d = 1: host copy of the cell-edge probabilities
  std::vector<int64_t> band_off;  // d = 1: banded stratified counts, row offsets [R + 1]
  std::vector<int32_t> band_lo;   // d = 1: first band column of every row [R]
  int32_t gt_Kmax = -1;           // d = 1: largest guide K over the layers (-1: no tables)
  int32_t gt_Bmax = 1;            // d = 1: largest guide table
  int64_t batch_chunks = 0;      // scratch chunks per layer per pass
  bool two_pass_ok = false;       // the workspace holds two-pass scratch
  bool two_pass_shape = false;    // the count blocks and LDS allow two-pass counting
  hipEvent_t trace_keys = nullptr;
  // stream and events of the overlapped histogram passes (made on first use)
  static constexpr int kMaxGroups = 8;
  mutable hipStream_t aux = nullptr;
  mutable hipEvent_t fork[kMaxGroups] = {};
  mutable hipEvent_t join = nullptr;

  ~qtree_plan() {
    if (aux) (void)hipStreamSynchronize(aux);
    for (hipEvent_t& e : fork)
      if (e) (void)hipEventDestroy(e);
    if (join) (void)hipEventDestroy(join);
    if (aux) (void)hipStreamDestroy(aux);
  }
};

namespace qtree {
// Record a failure for qtree_last_error and return its status.
qtree_status set_error(qtree_status s, const std::string& msg);

// Scratch of the two-pass counting: keys and segment starts for `chunks`
// chunks per layer per pass, and the most layer groups a call may use.
struct CountScratch {
  uint16_t* keys = nullptr;
  uint32_t* segs = nullptr;
  int64_t chunks = 0;
  int max_groups = 1;
};
qtree_status transitions_on_scratch(const qtree_plan* plan, uint64_t m0, uint64_t M,
                                    uint64_t seed, uint32_t contract_id, qtree_mode mode,
                                    int32_t* counts, void* stream, void* base, size_t bytes);
}  // namespace qtree

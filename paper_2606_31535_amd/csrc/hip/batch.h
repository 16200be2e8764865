// Grouped execution of many factors' sweeps (shared by the batched and the
// served forms): the argument blocks, per-step item maps and step list of a
// set of (factor, query plan, output) entries.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "device_handle.h"
#include "sweep_kernels.h"

namespace peers {

struct BatchEntry {
  FactorHandle* F = nullptr;
  const DeviceQueryPlan* plan = nullptr;
  double* R_dev = nullptr;  // results of the entry's plan (device)
  // partial slots and staging of this entry; null = the factor's own
  // workspace (the served form gives every batch workspaces of its own)
  double* part = nullptr;
  double* stage = nullptr;
};

struct BatchStage {
  int kind;
  int64_t off, n, grid;
};

// Candidate schedules of the bottom step (order of subtree work items and grid form).
constexpr int kBatchSchedules = 4;
extern const char* const kBatchScheduleNames[kBatchSchedules];

struct BatchLayout {
  std::vector<FactorArgs> fargs;
  std::vector<GroupItem> items;  // every step's items, then the bottom items of each schedule
  std::vector<BatchStage> stages;
  int bottom_stage = -1;
  int64_t bottom_off[kBatchSchedules] = {0, 0, 0, 0};
  int64_t bottom_grid[kBatchSchedules] = {0, 0, 0, 0};
  int64_t bottom_n = 0;
  uint64_t items_offset = 0;  // byte offset of the items after the argument blocks
  uint64_t bytes = 0;         // device bytes of argument blocks + items
  void use_schedule(int c);
};

// Builds the steps of the entries' sweeps (top tree, bottom subtrees, finish),
// with workspace pointers taken from each factor (they must be sized already).
void batch_layout(const DeviceHandle& D, const std::vector<BatchEntry>& E, BatchLayout& L);
// Copies argument blocks and items to `mem` (at least L.bytes) on stream s.
Status batch_upload(const BatchLayout& L, void* mem, hipStream_t s);
// Launches every step on stream s (mem as uploaded).
Status batch_launch(const BatchLayout& L, void* mem, hipStream_t s);
Status batch_launch_stage(const BatchLayout& L, const BatchStage& st, void* mem, hipStream_t s);

// One factor's sweep over a plan that reads only some top chains: the steps
// run as grouped launches restricted to those chains' items.
Status run_sweep_pruned(FactorHandle& F, DeviceQueryPlan& D, double* R_dev, hipStream_t s, bool profile,
                        const SweepWork* work = nullptr);

}  // namespace peers

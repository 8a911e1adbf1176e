// Host-side state of a grid handle (private to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sl.h"
#include "sl_device.h"

struct sl_prof_pair {
  int kind;  // 0 trajectories, 1 reconstruction, 2 limiter order words, 3 source terms
  hipEvent_t start, stop;
};

struct sl_grid {
  sl_grid_desc desc;
  std::vector<double> modes;
  sl::GridArgs g;
  sl::VelArgs v;
  int64_t ntot;
  size_t off_stats, off_disp, off_flags, off_ord, off_disp2, ws_bytes;
  // Source terms: lattice values and stage fields (nfields arrays of the value
  // precision each) and the RK registers of positions (2 FP64 planes) and
  // values (3), all per node.
  size_t off_src_h, off_src_g, off_src_qx, off_src_qh;
  // Per-axis sin/cos table of the fused trajectories (sl::trig_table_kernel);
  // 0 when the velocity family does not use one.
  size_t off_trig, trig_bytes;
  bool limiter_words;  // limiter order words from a separate pass
  int steps_since_reset;
  int64_t steps_launched, reconstructs_launched;
  // Kernel timing with events attached to the dispatch packets of every
  // prof_period-th launch of each kind (0: off).
  int prof_period;
  int64_t prof_count[4];
  std::vector<hipEvent_t> ev_free;
  std::vector<sl_prof_pair> pending;
  double prof_ms[4];
  int64_t prof_n[4];
};


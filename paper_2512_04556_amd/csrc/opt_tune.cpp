// Built-in launch table of the persistent optimiser: the work-group size and
// the resident work-groups per compute unit for a batch, by its size, its
// largest side and its largest tap count.  The rows are written by the
// project's autotuner (paper_2512_04556_amd/autotune.py), which times every
// candidate shape on seeded batches of each bucket and keeps the fastest.
#include "internal.hpp"

namespace disk {

namespace {
struct TuneRow {
    int max_B;          // the row applies to batches of at most this many targets
    int max_side_upto;  // ... whose largest side is at most this
    int max_T_upto;     // ... and whose largest tap count (all layers) is at most this
    int threads;
    int wgs_per_cu;
};
#include "opt_tune_table.inc"
}  // namespace

disk_opt_tune opt_default_tune(const disk_batch_meta& m) {
    for (const TuneRow& r : kTuneRows)
        if (m.B <= r.max_B && m.max_side <= r.max_side_upto && m.max_T <= r.max_T_upto)
            return disk_opt_tune{r.threads, r.wgs_per_cu};
    return disk_opt_tune{256, 4};
}

}  // namespace disk

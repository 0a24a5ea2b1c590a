// Built-in launch table of the persistent optimiser: resident work-groups per
// compute unit for a batch, by the batch's maximum side and size.  The rows
// are written by the project's autotuner (paper_2512_04556_amd/autotune.py),
// which times each candidate on seeded batches of the side bucket and keeps
// the fastest.
#include "internal.hpp"

namespace disk {

namespace {
struct TuneRow {
    int max_side_upto;   // the row applies to batches whose largest side is at most this
    int wgs_per_cu;
};
#include "opt_tune_table.inc"
}  // namespace

int opt_default_wgs_per_cu(const disk_batch_meta& m) {
    for (const TuneRow& r : kTuneRows)
        if (m.max_side <= r.max_side_upto) return r.wgs_per_cu;
    return 4;
}

}  // namespace disk

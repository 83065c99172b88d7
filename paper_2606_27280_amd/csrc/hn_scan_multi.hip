// Multi-database scans: dispatch by precision to the per-precision units.
#include "hn_scan.h"

namespace hn {
int launch_scan_multi(int precision, int mode, int w, int cfg, const ScanArgs *dbs,
                      const int2 *items, int n_items, const int *redo,
                      const unsigned *redo_count, unsigned *item_ctr, hipStream_t s) {
    switch (precision) {
        case HN_PREC_FP32:
            return launch_scan_multi_f32(mode, w, cfg, dbs, items, n_items, redo, redo_count,
                                         item_ctr, s);
        case HN_PREC_BF16:
            return launch_scan_multi_bf16(mode, w, cfg, dbs, items, n_items, redo, redo_count,
                                         item_ctr, s);
        case HN_PREC_FP8:
            return launch_scan_multi_fp8(mode, w, cfg, dbs, items, n_items, redo, redo_count,
                                         item_ctr, s);
        case HN_PREC_INT8:
            return launch_scan_multi_i8(mode, w, cfg, dbs, items, n_items, redo, redo_count,
                                         item_ctr, s);
    }
    return 1;
}
}  // namespace hn

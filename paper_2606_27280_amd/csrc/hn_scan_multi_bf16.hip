// Multi-database scan kernels for the bf16 streams (one launch over the
// work items of many databases of one stream width).
#include "hn_scan.h"

namespace hn {
int launch_scan_multi_bf16(int mode, int w, int cfg, const ScanArgs *dbs, const int2 *items,
                         int n_items, const int *redo, const unsigned *redo_count,
                         unsigned *item_ctr, hipStream_t s) {
#define HN_MULTI(Tile) \
    launch_tile_multi<Tile>(mode, cfg, dbs, items, n_items, redo, redo_count, item_ctr, s)
    switch (w) {
        case 16: return HN_MULTI(BF16Tile32<16>);
        case 32: return HN_MULTI(BF16Tile32<32>);
    }
#undef HN_MULTI
    return 1;
}
}  // namespace hn

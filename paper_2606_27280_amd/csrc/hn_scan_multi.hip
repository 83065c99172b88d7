// Multi-database scan kernels: one launch over the work items of many
// databases of the same stream width.
#include "hn_scan.h"

namespace hn {
int launch_scan_multi(int precision, int mode, int w, int cfg, const ScanArgs *dbs,
                      const int2 *items, int n_items, const int *redo,
                      const unsigned *redo_count, hipStream_t s) {
#define HN_MULTI(Tile) launch_tile_multi<Tile>(mode, cfg, dbs, items, n_items, redo, redo_count, s)
    if (precision == HN_PREC_FP32) {
        switch (w) {
            case 8: return HN_MULTI(F32Tile32<8>);
            case 16: return HN_MULTI(F32Tile32<16>);
            case 32: return HN_MULTI(F32Tile32<32>);
        }
    } else if (precision == HN_PREC_BF16) {
        switch (w) {
            case 16: return HN_MULTI(BF16Tile32<16>);
            case 32: return HN_MULTI(BF16Tile32<32>);
        }
    } else if (precision == HN_PREC_FP8) {
        switch (w) {
            case 16: return HN_MULTI(FP8Tile32<16>);
            case 32: return HN_MULTI(FP8Tile32<32>);
        }
    } else if (precision == HN_PREC_INT8) {
        switch (w) {
            case 16: return HN_MULTI(I8Tile32<16>);
            case 32: return HN_MULTI(I8Tile32<32>);
        }
    }
#undef HN_MULTI
    return 1;
}
}  // namespace hn

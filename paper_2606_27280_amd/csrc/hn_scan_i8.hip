// INT8 fixed-point scan kernels: widths 16 and 32 on the 32x32x16 int8 MFMA.
#include "hn_scan.h"

namespace hn {
int launch_scan_int8(int mode, int w, int cfg, const Plan &p, const ScanArgs &A, hipStream_t s) {
    switch (w) {
        case 16: return launch_tile<I8Tile32<16>, true>(mode, cfg, p, A, s);
        case 32: return launch_tile<I8Tile32<32>, true>(mode, cfg, p, A, s);
    }
    return 1;
}
unsigned slots_scan_int8(int mode, int w, int cfg) {
    switch (w) {
        case 16: return tile_slots<I8Tile32<16>, true>(mode, cfg);
        case 32: return tile_slots<I8Tile32<32>, true>(mode, cfg);
    }
    return 0;
}
}  // namespace hn

// Float32 scan kernels for stream widths 4, 8, 16 and 32 (K <= 32) on the
// 32x32x2 MFMA shape.
#include "hn_scan.h"

namespace hn {
int launch_scan_f32_narrow(int mode, int w, int cfg, const Plan &p, const ScanArgs &A,
                           hipStream_t s) {
    switch (w) {
        case 4: return launch_tile<F32Tile32<4>, true>(mode, cfg, p, A, s);
        case 8: return launch_tile<F32Tile32<8>, true>(mode, cfg, p, A, s);
        case 16: return launch_tile<F32Tile32<16>, true>(mode, cfg, p, A, s);
        case 32: return launch_tile<F32Tile32<32>, true>(mode, cfg, p, A, s);
    }
    return 1;
}
unsigned slots_scan_f32_narrow(int mode, int w, int cfg) {
    switch (w) {
        case 4: return tile_slots<F32Tile32<4>, true>(mode, cfg);
        case 8: return tile_slots<F32Tile32<8>, true>(mode, cfg);
        case 16: return tile_slots<F32Tile32<16>, true>(mode, cfg);
        case 32: return tile_slots<F32Tile32<32>, true>(mode, cfg);
    }
    return 0;
}
}  // namespace hn

// Float32 scan kernels for stream widths 64 and 128 on the 16x16x4 MFMA shape,
// including the exhaustive 128-wide scan and its window mode.
#include "hn_scan.h"

namespace hn {
int launch_scan_f32_wide(int mode, int w, int cfg, const Plan &p, const ScanArgs &A,
                         hipStream_t s) {
    switch (w) {
        case 64: return launch_tile<F32Tile<64>, true>(mode, cfg, p, A, s);
        case 128: return launch_tile<F32Tile<128>, true>(mode, cfg, p, A, s);
    }
    return 1;
}
unsigned slots_scan_f32_wide(int mode, int w, int cfg) {
    switch (w) {
        case 64: return tile_slots<F32Tile<64>, true>(mode, cfg);
        case 128: return tile_slots<F32Tile<128>, true>(mode, cfg);
    }
    return 0;
}
}  // namespace hn

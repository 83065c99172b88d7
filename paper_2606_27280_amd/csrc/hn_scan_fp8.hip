// FP8 (E4M3FN) scan kernels: widths 16 and 32, decoded to bf16 in registers
// for the 32x32x16 MFMA shape.
#include "hn_scan.h"

namespace hn {
int launch_scan_fp8(int mode, int w, int cfg, const Plan &p, const ScanArgs &A, hipStream_t s) {
    switch (w) {
        case 16: return launch_tile<FP8Tile32<16>, true>(mode, cfg, p, A, s);
        case 32: return launch_tile<FP8Tile32<32>, true>(mode, cfg, p, A, s);
    }
    return 1;
}
unsigned slots_scan_fp8(int mode, int w, int cfg) {
    switch (w) {
        case 16: return tile_slots<FP8Tile32<16>, true>(mode, cfg);
        case 32: return tile_slots<FP8Tile32<32>, true>(mode, cfg);
    }
    return 0;
}
}  // namespace hn

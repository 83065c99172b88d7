// Bfloat16 scan kernels: widths 16 and 32 on the 32x32x16 MFMA shape, widths
// 64 and 128 on 16x16x32.
#include "hn_scan.h"

namespace hn {
int launch_scan_bf16(int mode, int w, int cfg, const Plan &p, const ScanArgs &A, hipStream_t s) {
    switch (w) {
        case 16: return launch_tile<BF16Tile32<16>, true>(mode, cfg, p, A, s);
        case 32: return launch_tile<BF16Tile32<32>, true>(mode, cfg, p, A, s);
        case 64: return launch_tile<BF16Tile<64>, true>(mode, cfg, p, A, s);
        case 128: return launch_tile<BF16Tile<128>, true>(mode, cfg, p, A, s);
    }
    return 1;
}
unsigned slots_scan_bf16(int mode, int w, int cfg) {
    switch (w) {
        case 16: return tile_slots<BF16Tile32<16>, true>(mode, cfg);
        case 32: return tile_slots<BF16Tile32<32>, true>(mode, cfg);
        case 64: return tile_slots<BF16Tile<64>, true>(mode, cfg);
        case 128: return tile_slots<BF16Tile<128>, true>(mode, cfg);
    }
    return 0;
}
}  // namespace hn

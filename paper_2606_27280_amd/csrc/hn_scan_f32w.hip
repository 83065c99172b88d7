// Float32 scan kernels, stream widths 32, 64 and 128 (K > 16, and the
// exhaustive 128-wide scan with its window mode).
#include "hn_scan.h"

namespace hn {
int launch_scan_f32_wide(int mode, int w, int cfg, const Plan &p, const ScanArgs &A,
                         hipStream_t s) {
    switch (w) {
        case 32: return launch_tile<F32Tile<32>, false>(mode, cfg, p, A, s);
        case 64: return launch_tile<F32Tile<64>, false>(mode, cfg, p, A, s);
        case 128: return launch_tile<F32Tile<128>, true>(mode, cfg, p, A, s);
    }
    return 1;
}
}  // namespace hn

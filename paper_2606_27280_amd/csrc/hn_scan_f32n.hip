// Float32 scan kernels, stream widths 4, 8 and 16 (K <= 16).
#include "hn_scan.h"

namespace hn {
int launch_scan_f32_narrow(int mode, int w, int cfg, const Plan &p, const ScanArgs &A,
                           hipStream_t s) {
    switch (w) {
        case 4: return launch_tile<F32Tile<4>, false>(mode, cfg, p, A, s);
        case 8: return launch_tile<F32Tile<8>, false>(mode, cfg, p, A, s);
        case 16: return launch_tile<F32Tile<16>, false>(mode, cfg, p, A, s);
    }
    return 1;
}
}  // namespace hn

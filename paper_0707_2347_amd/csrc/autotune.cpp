// Choice of schedule, Winograd depth and base kind.
#include "wsmul_internal.hpp"

namespace wsmul {

int autotune_choice(ws_args &a, bool beta_nonzero) {
    if (a.schedule == WS_AUTO)
        a.schedule = WS_TWO_TEMP;
    if (a.levels < 0) {
        int64_t s = std::min(a.m, std::min(a.k, a.n));
        int l = 0;
        while (s >= 4096 && l < 4) {
            s /= 2;
            ++l;
        }
        a.levels = l;
    }
    (void)beta_nonzero;
    return WS_OK;
}

}  // namespace wsmul

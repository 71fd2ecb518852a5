// scan_i8_full.hip -- int8 MFMA, full H and p
#include "scan_kernel.h"

extern "C" hipError_t kx_scan_i8_full(const kx::ScanArgs* a, int ks, int grid, hipStream_t st) {
    using namespace kx;
    switch (ks) {
        case 1: return launch_one<I8, 1, MISS3, FULL>(*a, grid, st);
        case 2: return launch_one<I8, 2, MISS3, FULL>(*a, grid, st);
        case 3: return launch_one<I8, 3, MISS3, FULL>(*a, grid, st);
        case 4: return launch_one<I8, 4, MISS3, FULL>(*a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

// scan_f16_miss.hip -- fp16 MFMA, SNP tiles with missing genotypes, screen mode
#include "scan_kernel.h"

extern "C" hipError_t kx_scan_f16_miss(const kx::ScanArgs* a, int ks, int grid, hipStream_t st) {
    using namespace kx;
    switch (ks) {
        case 1: return launch_one<F16, 1, MISS3, SCREEN>(*a, grid, st);
        case 2: return launch_one<F16, 2, MISS3, SCREEN>(*a, grid, st);
        case 3: return launch_one<F16, 3, MISS3, SCREEN>(*a, grid, st);
        case 4: return launch_one<F16, 4, MISS3, SCREEN>(*a, grid, st);
        case 5: return launch_one<F16, 5, MISS3, SCREEN>(*a, grid, st);
        case 6: return launch_one<F16, 6, MISS3, SCREEN>(*a, grid, st);
        case 7: return launch_one<F16, 7, MISS3, SCREEN>(*a, grid, st);
        case 8: return launch_one<F16, 8, MISS3, SCREEN>(*a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

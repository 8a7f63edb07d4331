// Range compression kernels: per row, forward transform, product with the
// conjugate spectrum of the pulse replica, backward transform -- one
// LDS-resident workgroup per row (or rows), one read and one write of HBM.
#include "fft_kernel.hpp"

namespace fb {

#define FB_FLT(DEF, FL, N, E, C, ...)                                                          \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolFilt, FL>(DEF, "range_compress<" #N ",[" #__VA_ARGS__ \
                                                               "],v" #FL ">")

static const KEntry kFilter[] = {
    FB_FLT(true, 0, 64, 16, 64, 16, 4),
    FB_FLT(true, 0, 128, 16, 32, 16, 8),
    FB_FLT(true, 35, 256, 16, 16, 16, 16),
    FB_FLT(true, 35, 512, 8, 4, 8, 8, 8),
    FB_FLT(false, 35, 512, 16, 8, 16, 16, 2),
    FB_FLT(false, 35, 1024, 8, 2, 8, 8, 4, 4),
    FB_FLT(false, 35, 2048, 16, 2, 16, 16, 8),
    FB_FLT(true, 35, 4096, 16, 1, 16, 16, 16),
    FB_FLT(false, 35, 8192, 16, 1, 8, 8, 8, 16),
    FB_FLT(false, 35, 16384, 16, 1, 16, 16, 16, 4),
    // first radix equal to the last: no LDS round trip between the transforms
    // (measured faster at 1024, 2048, 8192 and 16384)
    FB_FLT(true, 35, 1024, 16, 4, 16, 4, 16),
    FB_FLT(false, 547, 1024, 16, 4, 16, 4, 16),
    FB_FLT(false, 547, 512, 16, 8, 16, 16, 2),
    FB_FLT(false, 35, 8192, 16, 1, 16, 8, 4, 16),
    FB_FLT(false, 35, 8192, 16, 1, 16, 2, 16, 16),
    FB_FLT(false, 43, 8192, 16, 1, 16, 2, 16, 16),
    FB_FLT(false, 35, 8192, 32, 1, 16, 32, 16),
    FB_FLT(false, 35, 8192, 32, 1, 32, 8, 32),
    FB_FLT(false, 35, 16384, 32, 1, 32, 16, 32),
    FB_FLT(true, 35, 2048, 16, 2, 16, 8, 16),
    FB_FLT(true, 35, 16384, 16, 1, 16, 4, 16, 16),
    FB_FLT(false, 3, 8192, 16, 1, 8, 8, 8, 16),
    // half exchanges (thirty-two values per thread, first radix = last): half
    // the LDS, four workgroups per CU instead of two at 8192 (67.6 against
    // 72.7 us for 2^24 points); slower at 4096 (68.5 / 62.8) and 16384
    // (100.9 / 89.0), where the registers, not the LDS, set the residency
    FB_FLT(false, 1059, 8192, 32, 1, 16, 8, 4, 16),
    FB_FLT(true, 1059, 8192, 32, 1, 16, 16, 2, 16),
    FB_FLT(false, 3107, 8192, 32, 1, 16, 16, 2, 16),
    FB_FLT(false, 1059, 4096, 32, 1, 16, 16, 16),
    FB_FLT(false, 1059, 16384, 32, 1, 16, 4, 16, 16),
};

const KEntry* filter_entries(int* count)
{
    *count = (int)(sizeof(kFilter) / sizeof(kFilter[0]));
    return kFilter;
}

}  // namespace fb

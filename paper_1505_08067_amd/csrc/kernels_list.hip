// List forms of the default block kernels: the same schedules and workgroup
// shapes, with each transform's source and destination read from a
// descriptor, so same-length requests anywhere in memory share one launch.
#include "fft_kernel.hpp"

namespace fb {

#define FB_LST(FL, N, E, C, ...) \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolList, FL>(true, "block_fft_list<" #N ",[" #__VA_ARGS__ "],v" #FL ">")

static const KEntry kList[] = {
    FB_LST(0, 2, 2, 256, 2),
    FB_LST(0, 4, 4, 256, 4),
    FB_LST(0, 8, 8, 256, 8),
    FB_LST(0, 16, 16, 256, 16),
    FB_LST(0, 32, 16, 128, 16, 2),
    FB_LST(0, 64, 16, 64, 16, 4),
    FB_LST(0, 128, 16, 32, 16, 8),
    FB_LST(35, 256, 16, 16, 16, 16),
    FB_LST(35, 512, 8, 4, 8, 8, 8),
    FB_LST(35, 1024, 16, 4, 16, 16, 4),
    FB_LST(35, 2048, 16, 2, 16, 16, 8),
    FB_LST(35, 4096, 16, 1, 16, 16, 16),
    FB_LST(1059, 8192, 32, 1, 8, 8, 8, 16),
    FB_LST(1059, 16384, 32, 1, 16, 4, 16, 16),
    FB_LST(0, 3, 3, 64, 3),
    FB_LST(0, 5, 5, 64, 5),
    FB_LST(0, 6, 6, 64, 6),
    FB_LST(0, 10, 10, 64, 10),
    FB_LST(0, 12, 12, 64, 12),
    FB_LST(0, 15, 15, 64, 15),
    FB_LST(0, 20, 20, 64, 20),
    FB_LST(0, 60, 30, 32, 6, 10),
    FB_LST(0, 100, 10, 8, 10, 10),
    FB_LST(0, 1000, 10, 2, 10, 10, 10),
    FB_LST(35, 3072, 24, 2, 6, 8, 8, 8),
    FB_LST(35, 6000, 30, 1, 10, 10, 10, 6),
    FB_LST(35, 15360, 60, 1, 12, 20, 4, 4, 4),
};

const KEntry* list_entries(int* count)
{
    *count = (int)(sizeof(kList) / sizeof(kList[0]));
    return kList;
}

}  // namespace fb

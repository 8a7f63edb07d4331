// Persistent ragged kernels, one per LDS-footprint class (see
// ragged_kernel.hpp).  A class shares one workgroup shape, one LDS size and
// one register budget; every case of a kernel must fit that budget without
// spilling (a kernel that uses scratch memory runs far below its occupancy),
// so lengths whose blocks need very different on-chip storage go to
// different kernels:
//
//   large : 1024 threads, up to 140 KB of LDS, 128 VGPRs, one workgroup per
//           CU -- 32768, two 16384-point transforms per workgroup, and pass 1
//           of the four-step lengths (64 columns of 256);
//   mid   : 256 threads, up to 35 KB, 168 VGPRs, three per CU or more -- 8192;
//   small : 256 threads, at most 35 KB and 128 VGPRs, four per CU -- every
//           length up to 4096, 1000, 3072 (12 values per thread, five
//           stages) and pass 2 of the four-step lengths (16 rows of 256).
//
// 6000 and 15360 have no case here, in either storage form: their own
// kernels, whose stages run on different thread counts (600 and 512 or 1024
// threads, at most 12 to 32 values per thread), beat any shared-footprint
// case (the FP16 fixed-E cases took 30 and 60 values per thread, the latter
// the whole register file), so the ragged plan runs them as plain launches
// beside the persistent ones.
//
// The launch holding four-step pass-1 tiles runs before the one holding the
// pass-2 tiles (the launch boundary orders the passes).  Each case equals a
// plain catalogue entry (same length, schedule, width and variant), whose
// plan builds the case's twiddle table.
#include "ragged_kernel.hpp"

namespace fb {

static const RKEntry kRagged[] = {
    make_rk_entry<256, 4,
                  RCase<64, 16, 64, Sched<16, 4>, PolBlock, 0>,
                  RCase<128, 16, 32, Sched<16, 8>, PolBlock, 0>,
                  RCase<256, 16, 16, Sched<16, 16>, PolBlock, 35>,
                  RCase<512, 16, 8, Sched<16, 16, 2>, PolBlock, 35>,
                  RCase<1024, 16, 4, Sched<16, 16, 4>, PolBlock, 35>,
                  RCase<2048, 16, 2, Sched<16, 16, 8>, PolBlock, 35>,
                  RCase<4096, 16, 1, Sched<16, 16, 16>, PolBlock, 35>,
                  RCase<1000, 10, 2, Sched<10, 10, 10>, PolBlock, 35>,
                  RCase<3072, 12, 1, Sched<12, 4, 4, 4, 4>, PolBlock, 35>,
                  RCase<256, 16, 16, Sched<16, 16>, PolPass2, 34>>("ragged_small_c64"),
    make_rk_entry<1024, 4,
                  RCase<32768, 32, 1, Sched<16, 8, 16, 16>, PolBlock, 1059>,
                  RCase<16384, 32, 2, Sched<16, 4, 16, 16>, PolBlock, 1059>,
                  RCase<256, 16, 64, Sched<16, 16>, PolPass1, 49>>("ragged_large_c64"),
    make_rk_entry<256, 3, RCase<8192, 32, 1, Sched<8, 8, 8, 16>, PolBlock, 1059>>("ragged_mid_c64"),
    // FP16 storage, FP32 arithmetic
    make_rk_entry<256, 4,
                  RCase<64, 16, 64, Sched<16, 4>, PolBlockH, 64>,
                  RCase<128, 16, 32, Sched<16, 8>, PolBlockH, 64>,
                  RCase<256, 16, 16, Sched<16, 16>, PolBlockH, 99>,
                  RCase<512, 16, 8, Sched<16, 16, 2>, PolBlockH, 99>,
                  RCase<1024, 16, 4, Sched<16, 16, 4>, PolBlockH, 99>,
                  RCase<2048, 16, 2, Sched<16, 16, 8>, PolBlockH, 99>,
                  RCase<4096, 16, 1, Sched<16, 16, 16>, PolBlockH, 99>,
                  RCase<1000, 10, 2, Sched<10, 10, 10>, PolBlockH, 64>,
                  RCase<3072, 12, 1, Sched<12, 4, 4, 4, 4>, PolBlockH, 99>,
                  RCase<256, 16, 16, Sched<16, 16>, PolPass2H, 98>>("ragged_small_f16"),
    make_rk_entry<1024, 4,
                  RCase<32768, 32, 1, Sched<16, 8, 16, 16>, PolBlockH, 1123>,
                  RCase<16384, 32, 2, Sched<16, 4, 16, 16>, PolBlockH, 1123>,
                  RCase<256, 16, 64, Sched<16, 16>, PolPass1H, 113>>("ragged_large_f16"),
    make_rk_entry<256, 3, RCase<8192, 32, 1, Sched<8, 8, 8, 16>, PolBlockH, 1131>>("ragged_mid_f16"),
};

const RKEntry* ragged_entries(int* count)
{
    *count = (int)(sizeof(kRagged) / sizeof(kRagged[0]));
    return kRagged;
}

}  // namespace fb

// Single-block kernels: one LDS-resident transform per group of N/E threads
// (paper, Approach: the elementary FFT block sized to one compute unit's
// local memory; "Top level analysis": read, compute, write).  Small lengths
// pack several transforms into one workgroup so it has at least one wave64.
//
// Each entry is one compiled (length, schedule, workgroup shape, variant);
// the entry marked default is the planner's choice, the others are there for
// the runtime sweep and the schedule search.
#include "fft_kernel.hpp"

namespace fb {

#define FB_BLK(DEF, FL, N, E, C, ...)                                                           \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolBlock, FL>(DEF, "block_fft<" #N ",[" #__VA_ARGS__ \
                                                                "],v" #FL ">")

// the same, with the workgroup width in the name (narrow variants of a
// schedule that also exists at full width)
#define FB_BLKC(DEF, FL, N, E, C, ...)                                                                  \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolBlock, FL>(DEF, "block_fft<" #N ",C" #C ",[" #__VA_ARGS__ \
                                                                "],v" #FL ">")

#define FB_BLKH(DEF, FL, N, E, C, ...)                                                               \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolBlockH, FL>(DEF, "block_fft_f16<" #N ",[" #__VA_ARGS__ \
                                                                 "],v" #FL ">")
#define FB_BLKHC(DEF, FL, N, E, C, ...)                                                                      \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolBlockH, FL>(DEF, "block_fft_f16<" #N ",C" #C ",[" #__VA_ARGS__ \
                                                                 "],v" #FL ">")

static const KEntry kBlock[] = {
    // wave-synchronous exchanges (whole transforms per wavefront, no barriers)
    FB_BLK(false, 547, 32, 16, 128, 16, 2),
    FB_BLK(false, 547, 64, 16, 64, 16, 4),
    FB_BLK(false, 547, 128, 16, 32, 16, 8),
    FB_BLK(false, 547, 256, 16, 16, 16, 16),
    FB_BLK(false, 547, 512, 16, 8, 16, 16, 2),
    FB_BLK(false, 547, 1024, 16, 4, 16, 16, 4),
    // thirty-two values per thread: one exchange fewer
    FB_BLK(false, 35, 8192, 32, 1, 16, 32, 16),
    FB_BLK(false, 35, 8192, 32, 1, 32, 8, 32),
    FB_BLK(false, 35, 16384, 32, 1, 32, 16, 32),
    // half exchanges at 4096 (eight workgroups per CU instead of four): no gain
    FB_BLK(false, 1059, 4096, 32, 1, 16, 16, 16),
    // other 32768 schedules (half exchanges)
    FB_BLK(false, 1059, 32768, 32, 1, 16, 16, 8, 16),
    FB_BLK(false, 1059, 32768, 32, 1, 8, 16, 16, 16),
    // cases of the persistent ragged kernels that are no planner default:
    // two 16384-point transforms per 1024-thread workgroup (half exchanges;
    // alone 66.8 against 55.2 us per 2^24 points for the 512-thread default,
    // one workgroup per CU against two, but within the persistent launch no
    // slower than a plain 16384 node beside it), 3072 with twelve values per
    // thread (one 256-thread transform, five stages), and the FP16 forms of
    // these and of the 256-thread 512 block
    FB_BLKC(false, 1059, 16384, 32, 2, 16, 4, 16, 16),
    FB_BLK(false, 35, 3072, 12, 1, 12, 4, 4, 4, 4),
    FB_BLKHC(false, 1123, 16384, 32, 2, 16, 4, 16, 16),
    FB_BLKH(false, 99, 3072, 12, 1, 12, 4, 4, 4, 4),
    FB_BLKH(false, 99, 512, 16, 8, 16, 16, 2),
    // persistent workgroups looping over units (no prefetch)
    FB_BLK(false, 4131, 4096, 16, 1, 16, 16, 16),
    // sixteen-byte global accesses (lane pairs exchanging halves by DPP)
    FB_BLK(false, 16419, 4096, 16, 1, 16, 16, 16),
    FB_BLK(false, 16419, 2048, 16, 2, 16, 16, 8),
    FB_BLK(false, 16419, 1024, 16, 4, 16, 16, 4),
    FB_BLK(false, 16419, 256, 16, 16, 16, 16),
    FB_BLK(false, 17443, 8192, 32, 1, 8, 8, 8, 16),
    // the schedule of the cross-lane 1024 kernels, with LDS exchanges
    FB_BLK(false, 35, 1024, 16, 4, 16, 4, 16),
    FB_BLK(false, 547, 1024, 16, 4, 16, 4, 16),
    // eight values per thread: twice the waves per workgroup at the same LDS
    FB_BLK(false, 35, 8192, 8, 1, 8, 8, 8, 8, 2),
    FB_BLK(false, 35, 2048, 8, 2, 8, 8, 4, 8),
    // FP16 storage, FP32 arithmetic (64 + 35; plain 64 where streaming hints
    // hurt: few threads per transform, so one load instruction spans many lines)
    FB_BLKH(true, 64, 2, 2, 256, 2),
    FB_BLKH(true, 64, 4, 4, 256, 4),
    FB_BLKH(true, 64, 8, 8, 256, 8),
    FB_BLKH(true, 64, 16, 16, 256, 16),
    FB_BLKH(true, 64, 32, 16, 128, 16, 2),
    FB_BLKH(true, 64, 64, 16, 64, 16, 4),
    FB_BLKH(true, 64, 128, 16, 32, 16, 8),
    FB_BLKH(true, 99, 256, 16, 16, 16, 16),
    FB_BLKH(true, 99, 512, 8, 4, 8, 8, 8),
    FB_BLKH(true, 99, 1024, 16, 4, 16, 16, 4),
    FB_BLKH(true, 99, 2048, 16, 2, 16, 16, 8),
    FB_BLKH(true, 99, 4096, 16, 1, 16, 16, 16),
    // half exchanges (see the complex64 defaults): 8192 63.7 against 76 us,
    // 16384 66.7 against 81.7 us for 2^25 points
    FB_BLKH(true, 1131, 8192, 32, 1, 8, 8, 8, 16),
    FB_BLKH(false, 107, 8192, 16, 1, 8, 8, 8, 16),
    FB_BLKH(true, 1123, 16384, 32, 1, 16, 4, 16, 16),
    FB_BLKH(false, 99, 16384, 16, 1, 16, 4, 16, 16),
    FB_BLKH(true, 1123, 32768, 32, 1, 16, 8, 16, 16),
    FB_BLKH(true, 64, 3, 3, 64, 3),
    FB_BLKH(true, 64, 5, 5, 64, 5),
    FB_BLKH(true, 64, 6, 6, 64, 6),
    FB_BLKH(true, 64, 10, 10, 64, 10),
    FB_BLKH(true, 64, 12, 12, 64, 12),
    FB_BLKH(true, 64, 15, 15, 64, 15),
    FB_BLKH(true, 64, 20, 20, 64, 20),
    FB_BLKH(true, 64, 60, 30, 32, 6, 10),
    FB_BLKH(true, 64, 100, 10, 8, 10, 10),
    FB_BLKH(true, 64, 1000, 10, 2, 10, 10, 10),
    FB_BLKH(true, 99, 3072, 24, 2, 6, 8, 8, 8),
    FB_BLKH(false, 99, 6000, 30, 1, 10, 10, 10, 6),
    FB_BLKH(false, 99, 15360, 60, 1, 12, 20, 4, 4, 4),
    // planner defaults: non-temporal data access + power-row twiddles (35)
    FB_BLK(true, 0, 2, 2, 256, 2),
    FB_BLK(false, 3, 2, 2, 256, 2),
    FB_BLK(true, 0, 4, 4, 256, 4),
    FB_BLK(false, 3, 4, 4, 256, 4),
    FB_BLK(true, 0, 8, 8, 256, 8),
    FB_BLK(false, 3, 8, 8, 256, 8),
    FB_BLK(true, 0, 16, 16, 256, 16),
    FB_BLK(false, 3, 16, 16, 256, 16),
    FB_BLK(true, 0, 32, 16, 128, 16, 2),
    FB_BLK(false, 35, 32, 16, 128, 16, 2),
    FB_BLK(true, 0, 64, 16, 64, 16, 4),
    FB_BLK(false, 35, 64, 16, 64, 16, 4),
    FB_BLK(true, 0, 128, 16, 32, 16, 8),
    FB_BLK(false, 35, 128, 16, 32, 16, 8),
    FB_BLK(true, 35, 256, 16, 16, 16, 16),
    FB_BLK(true, 35, 512, 8, 4, 8, 8, 8),
    FB_BLK(false, 35, 512, 16, 8, 16, 16, 2),
    FB_BLK(false, 35, 1024, 16, 4, 16, 16, 4),
    FB_BLK(false, 35, 1024, 8, 2, 8, 8, 4, 4),
    FB_BLK(true, 35, 2048, 16, 2, 16, 16, 8),
    FB_BLK(true, 35, 4096, 16, 1, 16, 16, 16),
    // 8192 and 16384: 32 values per thread with half exchanges, so the LDS
    // of a workgroup halves (8192: four workgroups per CU instead of two,
    // 97 against 102 us for 2^25 points; 16384: two instead of one, 107.7
    // against 117.3 us, and 57.7 against 61.4 for 2^24; below 512
    // transforms the 16-value form is faster: 256 x 16.9 / 20.7 us)
    FB_BLK(true, 1059, 8192, 32, 1, 8, 8, 8, 16),
    FB_BLK(false, 43, 8192, 16, 1, 8, 8, 8, 16),
    FB_BLK(false, 35, 8192, 16, 1, 8, 8, 8, 16),
    FB_BLK(true, 1059, 16384, 32, 1, 16, 4, 16, 16),
    FB_BLK(false, 35, 16384, 16, 1, 16, 4, 16, 16),
    FB_BLK(false, 35, 16384, 16, 1, 16, 16, 16, 4),
    // 32768 in one workgroup: half exchanges need 16384 LDS slots (128 KiB),
    // one workgroup per CU; 141 against 179 us (four-step 256 x 128) for
    // 2^25 points
    FB_BLK(true, 1059, 32768, 32, 1, 16, 8, 16, 16),
    // mixed-radix lengths (radix 3 and 5 butterflies and their products)
    FB_BLK(true, 0, 3, 3, 64, 3),
    FB_BLK(false, 35, 3, 3, 64, 3),
    FB_BLK(true, 0, 5, 5, 64, 5),
    FB_BLK(false, 35, 5, 5, 64, 5),
    FB_BLK(true, 0, 6, 6, 64, 6),
    FB_BLK(false, 35, 6, 6, 64, 6),
    FB_BLK(true, 0, 10, 10, 64, 10),
    FB_BLK(false, 35, 10, 10, 64, 10),
    FB_BLK(true, 0, 12, 12, 64, 12),
    FB_BLK(false, 35, 12, 12, 64, 12),
    FB_BLK(true, 0, 15, 15, 64, 15),
    FB_BLK(false, 35, 15, 15, 64, 15),
    FB_BLK(true, 0, 20, 20, 64, 20),
    FB_BLK(false, 35, 20, 20, 64, 20),
    FB_BLK(true, 0, 60, 30, 32, 6, 10),
    FB_BLK(false, 35, 60, 30, 32, 6, 10),
    FB_BLK(true, 0, 100, 10, 8, 10, 10),
    FB_BLK(false, 35, 100, 10, 8, 10, 10),
    FB_BLK(true, 0, 1000, 10, 2, 10, 10, 10),
    FB_BLK(false, 35, 1000, 10, 2, 10, 10, 10),
    FB_BLK(true, 35, 3072, 24, 2, 6, 8, 8, 8),
    FB_BLK(false, 35, 6000, 30, 1, 10, 10, 10, 6),
    FB_BLK(false, 35, 15360, 60, 1, 12, 20, 4, 4, 4),
    FB_BLK(false, 3, 3072, 24, 2, 6, 8, 8, 8),
    FB_BLK(false, 0, 6000, 30, 1, 10, 10, 10, 6),
    FB_BLK(false, 3, 15360, 60, 1, 12, 20, 4, 4, 4),
    // plain variants (full twiddle rows, ordinary loads/stores)
    FB_BLK(false, 0, 256, 16, 16, 16, 16),
    FB_BLK(false, 0, 512, 16, 8, 16, 16, 2),
    FB_BLK(false, 0, 1024, 16, 4, 16, 16, 4),
    FB_BLK(false, 0, 2048, 16, 2, 16, 16, 8),
    FB_BLK(false, 0, 4096, 16, 1, 16, 16, 16),
    FB_BLK(false, 0, 8192, 32, 1, 32, 16, 16),
    FB_BLK(false, 0, 16384, 16, 1, 16, 16, 16, 4),
    // other variants of the main sizes: non-temporal (1|2), persistent with
    // LDS twiddles (4), swizzled LDS (8), power-row twiddles (32)
    FB_BLK(false, 3, 1024, 16, 4, 16, 16, 4),
    FB_BLK(false, 0, 1024, 8, 2, 8, 8, 4, 4),
    FB_BLK(false, 3, 1024, 8, 2, 8, 8, 4, 4),
    FB_BLK(false, 32, 1024, 8, 2, 8, 8, 4, 4),
    FB_BLK(false, 7, 1024, 8, 2, 8, 8, 4, 4),
    FB_BLK(false, 43, 1024, 8, 2, 8, 8, 4, 4),
    FB_BLK(false, 3, 4096, 16, 1, 16, 16, 16),
    FB_BLK(false, 32, 4096, 16, 1, 16, 16, 16),
    FB_BLK(false, 43, 4096, 16, 1, 16, 16, 16),
    FB_BLK(false, 7, 4096, 16, 1, 16, 16, 16),
    FB_BLK(false, 0, 4096, 8, 1, 8, 8, 8, 8),
    FB_BLK(false, 35, 4096, 8, 1, 8, 8, 8, 8),
    FB_BLK(false, 7, 4096, 8, 1, 8, 8, 8, 8),
    FB_BLK(false, 3, 8192, 32, 1, 32, 16, 16),
    FB_BLK(false, 35, 8192, 32, 1, 32, 16, 16),
    FB_BLK(false, 0, 8192, 16, 1, 8, 8, 8, 16),
    FB_BLK(false, 3, 16384, 16, 1, 16, 16, 16, 4),
    FB_BLK(false, 7, 16384, 16, 1, 16, 16, 16, 4),
    // alternative schedules (radix search)
    FB_BLK(false, 0, 512, 8, 4, 8, 8, 8),
    FB_BLK(false, 0, 1024, 16, 4, 4, 16, 16),
    FB_BLK(false, 0, 1024, 8, 2, 4, 8, 8, 4),
    FB_BLK(false, 35, 1024, 8, 2, 4, 8, 8, 4),
    FB_BLK(false, 0, 1024, 8, 2, 8, 8, 8, 2),
    FB_BLK(false, 35, 1024, 8, 2, 8, 8, 8, 2),
    FB_BLK(false, 0, 4096, 16, 1, 4, 16, 16, 4),
    FB_BLK(false, 0, 8192, 16, 1, 16, 16, 16, 2),
    FB_BLK(false, 0, 8192, 32, 1, 16, 16, 32),
    FB_BLK(false, 0, 16384, 32, 1, 32, 32, 16),
    FB_BLK(false, 35, 16384, 32, 1, 32, 32, 16),
    // small batches: one wavefront per workgroup (fewer transforms per
    // workgroup, same schedule and variant), so a batch too small to fill the
    // device spreads over more compute units; listed last so that a search by
    // schedule and variant alone finds the full-width kernel first
    FB_BLKC(false, 0, 16, 16, 64, 16),
    FB_BLKC(false, 0, 32, 16, 32, 16, 2),
    FB_BLKC(false, 0, 64, 16, 16, 16, 4),
    FB_BLKC(false, 0, 128, 16, 8, 16, 8),
    FB_BLKC(false, 35, 256, 16, 4, 16, 16),
    FB_BLKC(false, 35, 512, 8, 1, 8, 8, 8),
    FB_BLKC(false, 35, 1024, 16, 1, 16, 16, 4),
    FB_BLKC(false, 35, 2048, 16, 1, 16, 16, 8),
    FB_BLKC(false, 0, 1000, 10, 1, 10, 10, 10),
    FB_BLKC(false, 35, 3072, 24, 1, 6, 8, 8, 8),
};

const KEntry* block_entries(int* count)
{
    *count = (int)(sizeof(kBlock) / sizeof(kBlock[0]));
    return kBlock;
}

}  // namespace fb

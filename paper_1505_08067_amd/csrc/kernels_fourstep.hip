// Four-step passes for transforms longer than one LDS-resident block
// (paper, Approach, "Other FFT sizes": a larger FFT built from block-sized
// FFTs by splitting its stages, with more data exchange).  N = N1 * N2,
// input n = N2*n1 + n2, output k = k1 + N1*k2:
//
//   pass 1: the N1-point transform of every column n2 (C columns per
//           workgroup, so the strided reads move runs of C*8 bytes), each
//           output multiplied by exp(-2 pi i n2 k1 / N), stored to the
//           workspace in row blocks of CW (the pass-2 width): W[k1/CW][n2][k1%CW];
//   pass 2: the N2-point transform of every row k1 (CW rows per workgroup,
//           read contiguously), output k2 stored to X[k1 + N1*k2] -- the
//           corner turn fused into the store (runs of CW*8 bytes).
//
// The long twiddle exp(-2 pi i m / N), m = n2*k1 mod N, is the product of two
// small FP32 tables generated in FP64: hi[m >> b] * lo[m & (2^b - 1)].
#include "fft_kernel.hpp"

namespace fb {

#define FB_P1(DEF, FL, N, E, C, ...) \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolPass1, FL>(DEF, "fourstep_pass1<" #N ",C" #C ",[" #__VA_ARGS__ "],v" #FL ">")
#define FB_P2(DEF, FL, N, E, C, ...) \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolPass2, FL>(DEF, "fourstep_pass2<" #N ",C" #C ",[" #__VA_ARGS__ "],v" #FL ">")

#define FB_P1H(DEF, FL, N, E, C, ...) \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolPass1H, FL>(DEF, "fourstep_pass1_f16<" #N ",C" #C ",[" #__VA_ARGS__ "],v" #FL ">")
#define FB_P2H(DEF, FL, N, E, C, ...) \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolPass2H, FL>(DEF, "fourstep_pass2_f16<" #N ",C" #C ",[" #__VA_ARGS__ "],v" #FL ">")
// FP16 data and an FP16 workspace (FFT_STORAGE_F16_COMPACT)
#define FB_P1HW(DEF, FL, N, E, C, ...) \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolPass1HW, FL>(DEF, "fourstep_pass1_f16w<" #N ",C" #C ",[" #__VA_ARGS__ "],v" #FL ">")
#define FB_P2HW(DEF, FL, N, E, C, ...) \
    make_entry<N, E, C, Sched<__VA_ARGS__>, PolPass2HW, FL>(DEF, "fourstep_pass2_f16w<" #N ",C" #C ",[" #__VA_ARGS__ "],v" #FL ">")

static const KEntry kPass[] = {
    // narrower tiles (more workgroups per CU, half-line runs), plain and
    // XCD-ordered so the neighbouring tiles that complete a cache line run in
    // the same L2: measured slower than the defaults at 2^19..2^21
    // LDS stride residue shifted by 8 for the staged store (flag 256)
    FB_P1(false, 305, 512, 16, 16, 16, 16, 2),
    FB_P1(false, 305, 1024, 16, 16, 16, 16, 4),
    FB_P1(false, 305, 256, 16, 16, 16, 16),
    FB_P1(false, 305, 2048, 16, 8, 16, 16, 8),
    // 32 values per thread: one LDS exchange instead of two
    FB_P1(false, 49, 512, 32, 16, 32, 16),
    FB_P1(false, 177, 512, 16, 8, 16, 16, 2),
    FB_P1(false, 177, 1024, 16, 8, 16, 16, 4),
    FB_P2(false, 161, 2048, 16, 4, 16, 16, 8),
    // half exchanges through half the LDS: without streaming loads, and at
    // 128; pass 2 at 2048 with 32 values per thread and registers fitted to
    // two workgroups per CU (a few spilled): 52.4 against 53.0 us, within
    // the run-to-run spread, so not the default
    FB_P1(false, 1072, 512, 32, 16, 16, 32),
    FB_P1(false, 1073, 128, 16, 16, 8, 16),
    // 512: 32-column tiles (256-byte runs), and workgroups looping over tiles
    FB_P1(false, 1073, 512, 32, 32, 16, 32),
    FB_P1(false, 5169, 512, 32, 16, 16, 32),
    FB_P2(false, 3106, 2048, 32, 8, 16, 16, 8),
    FB_P2(false, 3362, 2048, 16, 8, 8, 8, 8, 4),
    // persistent workgroups looping over units (no prefetch, no spills)
    FB_P2(false, 4130, 2048, 16, 8, 16, 16, 8),
    // pass 2 reads the workspace pass 1 has just written (partly still in the
    // Infinity Cache): cached loads, power-row twiddles, with / without
    // streaming stores
    FB_P2(false, 32, 512, 16, 16, 16, 16, 2),
    FB_P2(false, 32, 1024, 16, 8, 16, 16, 4),
    FB_P2(false, 32, 2048, 16, 8, 16, 16, 8),
    FB_P2(false, 0, 512, 16, 16, 16, 16, 2),
    // FP16 storage (pass 1 reads FP16, pass 2 writes FP16; workspace FP32)
    FB_P1H(true, 113, 32, 16, 16, 16, 2),
    FB_P1H(true, 113, 64, 16, 16, 16, 4),
    FB_P1H(true, 113, 128, 16, 16, 16, 8),
    FB_P1H(false, 113, 256, 16, 16, 16, 16),
    FB_P1H(false, 113, 512, 16, 16, 16, 16, 2),
    FB_P1H(false, 113, 1024, 16, 16, 16, 16, 4),
    FB_P1H(false, 113, 2048, 16, 8, 16, 16, 8),
    // 32 FP16 columns = 128-byte runs; 16 FP16 rows = 64-byte output runs
    FB_P1H(false, 113, 256, 16, 32, 16, 16),
    FB_P1H(false, 113, 512, 16, 32, 16, 16, 2),
    FB_P2H(false, 98, 1024, 16, 16, 16, 16, 4),
    FB_P2H(true, 98, 32, 16, 16, 16, 2),
    FB_P2H(true, 98, 64, 16, 16, 16, 4),
    FB_P2H(true, 98, 128, 16, 16, 16, 8),
    FB_P2H(true, 98, 256, 16, 16, 16, 16),
    FB_P2H(false, 98, 512, 16, 16, 16, 16, 2),
    FB_P2H(false, 98, 1024, 16, 8, 16, 16, 4),
    FB_P2H(true, 98, 2048, 16, 8, 16, 16, 8),
    // 32 values per thread with half exchanges (69 KB of LDS, two workgroups
    // per CU; the 16-value forms hold all 16384 points of a workgroup in 139
    // KB, one per CU), pass 1 with registers fitted to two workgroups.  The
    // defaults at 1024 (1024 x 1024 at 2^20 x 16, forward, interleaved
    // medians): FP16 storage 98.0 against 110.8 us, compact form 75.3
    // against 90.9 us.  The 512 x 2048 split stays slower (FP16 output runs
    // of 8 rows are 32 bytes): 126 / 112 us.
    FB_P1H(false, 1137, 1024, 32, 16, 16, 16, 4),
    FB_P1H(true, 3185, 1024, 32, 16, 16, 16, 4),
    FB_P1HW(true, 527473, 1024, 32, 16, 16, 16, 4),
    // at 512 (2^19 x 32, 512 x 1024): 81.7 against 90.4 us, compact 59.6
    // against 73.1 us
    FB_P1H(true, 1137, 512, 32, 32, 16, 32),
    FB_P2H(true, 1122, 1024, 32, 16, 16, 16, 4),
    FB_P2H(false, 1122, 2048, 32, 8, 16, 16, 8),
    FB_P1HW(false, 525425, 1024, 32, 16, 16, 16, 4),
    FB_P1HW(true, 525425, 512, 32, 32, 16, 32),
    // pass 1 at 256 and pass 2 at 512 the same way (four workgroups per CU
    // instead of two): 2^18 x 64 77.1 against 80.3 us (compact 59.7 / 61.9),
    // 2^17 x 128 75.7 against 79.5 us (compact 56.4 / 59.2)
    FB_P1H(true, 1137, 256, 32, 32, 16, 16),
    FB_P1HW(true, 525425, 256, 32, 32, 16, 16),
    FB_P2H(true, 1122, 512, 32, 16, 16, 32),
    FB_P2HW(true, 525410, 512, 32, 16, 16, 32),
    FB_P2HW(true, 525410, 1024, 32, 16, 16, 16, 4),
    FB_P2HW(false, 525410, 2048, 32, 8, 16, 16, 8),
    // pass 1 at 2048 the same way (FP16 / compact, forward, 2^24 points):
    // 2^21 x 8 128.5 against 135.7 us / 110.0 against 118.7; 2^22 x 4 160.6
    // against 168.2 / 146.8 against 156.1.  Pass 2 at 2048 stays the
    // 16-value form (2^22 x 4 with both halved: 173.7 / 157.0 us).
    FB_P1H(true, 3185, 2048, 32, 8, 16, 16, 8),
    FB_P1HW(true, 527473, 2048, 32, 8, 16, 16, 8),
    // the same passes with an FP16 workspace: the defaults of the compact form
    FB_P1HW(true, 524401, 32, 16, 16, 16, 2),
    FB_P1HW(true, 524401, 64, 16, 16, 16, 4),
    FB_P1HW(true, 524401, 128, 16, 16, 16, 8),
    FB_P1HW(false, 524401, 256, 16, 32, 16, 16),
    FB_P1HW(false, 524401, 512, 16, 32, 16, 16, 2),
    FB_P1HW(false, 524401, 1024, 16, 16, 16, 16, 4),
    FB_P1HW(false, 524401, 2048, 16, 8, 16, 16, 8),
    FB_P2HW(true, 524386, 32, 16, 16, 16, 2),
    FB_P2HW(true, 524386, 64, 16, 16, 16, 4),
    FB_P2HW(true, 524386, 128, 16, 16, 16, 8),
    FB_P2HW(true, 524386, 256, 16, 16, 16, 16),
    FB_P2HW(false, 524386, 512, 16, 16, 16, 16, 2),
    FB_P2HW(false, 524386, 1024, 16, 16, 16, 16, 4),
    FB_P2HW(true, 524386, 2048, 16, 8, 16, 16, 8),
    // planner defaults.  Pass 1: non-temporal loads, power-row twiddles
    // (stage and long), outputs staged through LDS for contiguous stores
    // (49).  Pass 2: non-temporal loads, power-row twiddles (33).
    FB_P1(true, 49, 32, 16, 16, 16, 2),
    FB_P1(true, 49, 64, 16, 16, 16, 4),
    FB_P1(true, 49, 128, 16, 16, 16, 8),
    FB_P1(true, 49, 256, 16, 16, 16, 16),
    // 512: [16, 32] with half exchanges (35 KB of LDS, three workgroups per
    // CU instead of two: 51.8 against 56.3 us at 2^20 x 16, same results)
    FB_P1(true, 1073, 512, 32, 16, 16, 32),
    FB_P1(false, 49, 512, 32, 16, 16, 32),
    FB_P1(false, 49, 512, 16, 16, 16, 16, 2),
    FB_P1(false, 49, 1024, 16, 16, 16, 16, 4),
    // 32 values per thread with half exchanges: faster at 2^20 (1024 x 1024:
    // 65.9 against 69.6 us), slower at 2^21 (1024 x 2048: 71 against 67 us)
    FB_P1(false, 1073, 1024, 32, 16, 16, 16, 4),
    // the same with registers fitted to two workgroups per CU (124 VGPRs,
    // 69 KB of LDS; the 16-value form holds one 1024-thread workgroup per
    // CU): the defaults at 1024 and 2048.  Forward, cold, interleaved
    // medians: 2^21 x 8 (1024 x 2048) 108.7 against 117.6 us, 2^22 x 4
    // (2048 x 2048) 131.3 against 140.1 us
    FB_P1(true, 3121, 1024, 32, 16, 16, 16, 4),
    FB_P1(true, 3121, 2048, 32, 8, 16, 16, 8),
    FB_P1(false, 49, 2048, 16, 8, 16, 16, 8),
    // pass 2: cached loads of the workspace pass 1 has just written (partly
    // still in the Infinity Cache), streaming stores of the result
    FB_P2(true, 34, 32, 16, 16, 16, 2),
    FB_P2(true, 34, 64, 16, 16, 16, 4),
    FB_P2(true, 34, 128, 16, 16, 16, 8),
    FB_P2(true, 34, 256, 16, 16, 16, 16),
    FB_P2(true, 34, 512, 16, 16, 16, 16, 2),
    FB_P2(true, 34, 1024, 16, 8, 16, 16, 4),
    // 2048: 32 values per thread with half exchanges, 69 KB of LDS and 124
    // VGPRs, so two workgroups share a CU (47.3 against 50.9 us for
    // 2^20 x 16); the one-workgroup form stays as a variant
    FB_P2(true, 1058, 2048, 32, 8, 16, 16, 8),
    FB_P2(false, 34, 2048, 16, 8, 16, 16, 8),
    FB_P2(false, 33, 32, 16, 16, 16, 2),
    FB_P2(false, 33, 64, 16, 16, 16, 4),
    FB_P2(false, 33, 128, 16, 16, 16, 8),
    FB_P2(false, 33, 256, 16, 16, 16, 16),
    FB_P2(false, 33, 512, 16, 16, 16, 16, 2),
    FB_P2(false, 33, 1024, 16, 8, 16, 16, 4),
    FB_P2(false, 33, 2048, 16, 8, 16, 16, 8),
    // plain and other variants (1: nt load, 16: staged store, 32: power twiddles)
    FB_P1(false, 0, 1024, 16, 16, 16, 16, 4),
    FB_P1(false, 0, 1024, 16, 8, 16, 16, 4),
    FB_P1(false, 1, 1024, 16, 16, 16, 16, 4),
    FB_P1(false, 17, 1024, 16, 16, 16, 16, 4),
    FB_P1(false, 33, 1024, 16, 16, 16, 16, 4),
    FB_P1(false, 48, 1024, 16, 16, 16, 16, 4),
    FB_P1(false, 49, 1024, 16, 8, 16, 16, 4),
    FB_P1(false, 0, 2048, 16, 8, 16, 16, 8),
    FB_P2(false, 0, 1024, 16, 16, 16, 16, 4),
    FB_P2(false, 0, 1024, 16, 8, 16, 16, 4),
    FB_P2(false, 1, 1024, 16, 8, 16, 16, 4),
    FB_P2(false, 33, 1024, 16, 16, 16, 16, 4),
    FB_P2(false, 0, 2048, 16, 8, 16, 16, 8),
    // 64 columns of 256 per 1024-thread workgroup (512-byte runs): pass 1 of
    // the four-step lengths in the large persistent ragged kernel
    FB_P1(false, 49, 256, 16, 64, 16, 16),
    FB_P1H(false, 113, 256, 16, 64, 16, 16),
    // half-line tiles (found by explicit width only)
    FB_P1(false, 49, 512, 16, 8, 16, 16, 2),
    FB_P2(false, 33, 2048, 16, 4, 16, 16, 8),
};

const KEntry* pass_entries(int* count)
{
    *count = (int)(sizeof(kPass) / sizeof(kPass[0]));
    return kPass;
}

}  // namespace fb

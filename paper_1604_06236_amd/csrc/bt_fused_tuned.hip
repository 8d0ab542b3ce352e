// Alternative fused schedules (radix order, threads per block, blocks per
// workgroup) for the standard block shapes; the autotuner picks among these
// and the defaults.
#include <vector>

#include "bt_fused.hpp"

namespace bt {
void register_fused_tuned(std::vector<FusedEntry> &v)
{
    const FusedEntry e[] = {
        // K = 16, M = 5 (N = 80)
        make_entry<Radices<5, 16>, 16, 4>(16, 5),
        make_entry<Radices<5, 4, 4>, 32, 8>(16, 5),
        // K = 128, M = 15 (N = 1920)
        make_entry<Radices<15, 8, 16>, 128, 2>(128, 15),
        make_entry<Radices<15, 16, 8>, 256, 1>(128, 15),
        make_entry<Radices<15, 16, 8>, 64, 4>(128, 15),
        make_entry<Radices<15, 16, 8>, 128, 1>(128, 15),
        // K = 256, M = 9 (N = 2304)
        make_entry<Radices<9, 16, 16>, 128, 2>(256, 9),
        make_entry<Radices<9, 16, 16>, 256, 2>(256, 9),
        make_entry<Radices<9, 8, 32>, 256, 1>(256, 9),
        // K = 1024, M = 15 (N = 15360)
        make_entry<Radices<15, 16, 16, 4>, 1024, 1>(1024, 15),
        make_entry<Radices<15, 4, 16, 16>, 1024, 1>(1024, 15),
        make_entry<Radices<15, 16, 16, 4>, 512, 1>(1024, 15),
        make_entry<Radices<15, 16, 16, 4>, 1024, 1, OPT_NO_PREFETCH>(1024, 15),
        make_entry<Radices<15, 16, 16, 4>, 1024, 1, OPT_NO_PREFETCH | OPT_SEQ_TWIDDLE>(1024, 15),
        make_entry<Radices<15, 8, 8, 16>, 1024, 1, OPT_NO_PREFETCH | OPT_SEQ_TWIDDLE>(1024, 15),
        make_entry<Radices<15, 16, 16, 4>, 1024, 1, OPT_SEQ_TWIDDLE>(1024, 15),
        make_entry<Radices<15, 32, 32>, 512, 1, OPT_NO_PREFETCH | OPT_SEQ_TWIDDLE>(1024, 15),
        make_entry<Radices<15, 8, 8, 16>, 1024, 1, OPT_SEQ_TWIDDLE>(1024, 15),
        make_entry<Radices<15, 8, 8, 16>, 1024, 1, OPT_SEQ_TWIDDLE | OPT_NT>(1024, 15),
        // K = 128, M = 15 and K = 256, M = 9 with sequential twiddles
        make_entry<Radices<15, 16, 8>, 128, 1, OPT_SEQ_TWIDDLE>(128, 15),
        make_entry<Radices<9, 16, 16>, 256, 1, OPT_SEQ_TWIDDLE>(256, 9),
        // 16-byte I/O (two adjacent butterflies per thread at the HBM ends), non-temporal
        make_entry<Radices<15, 16, 8>, 64, 2, OPT_SEQ_TWIDDLE | OPT_PAIRED_IO>(128, 15),
        make_entry<Radices<15, 16, 8>, 64, 1, OPT_SEQ_TWIDDLE | OPT_PAIRED_IO>(128, 15),
        make_entry<Radices<15, 16, 8>, 128, 1, OPT_SEQ_TWIDDLE | OPT_NT>(128, 15),
        make_entry<Radices<15, 16, 8>, 64, 2, OPT_SEQ_TWIDDLE | OPT_PAIRED_IO | OPT_NT>(128, 15),
        make_entry<Radices<15, 8, 16>, 64, 2, OPT_SEQ_TWIDDLE | OPT_PAIRED_IO>(128, 15),
        make_entry<Radices<9, 16, 16>, 128, 2, OPT_SEQ_TWIDDLE | OPT_PAIRED_IO>(256, 9),
        make_entry<Radices<9, 16, 16>, 128, 1, OPT_SEQ_TWIDDLE | OPT_PAIRED_IO>(256, 9),
        make_entry<Radices<9, 16, 16>, 256, 1, OPT_SEQ_TWIDDLE | OPT_NT>(256, 9),
        make_entry<Radices<5, 4, 4>, 16, 8, OPT_PAIRED_IO>(16, 5),
        // non-temporal variants of the other plans
        make_entry<Radices<15, 32, 32>, 512, 1, OPT_NT>(1024, 15),
        make_entry<Radices<15, 32, 32>, 512, 1, OPT_SEQ_TWIDDLE | OPT_NT>(1024, 15),
        make_entry<Radices<15, 16, 16, 4>, 1024, 1, OPT_SEQ_TWIDDLE | OPT_NT>(1024, 15),
        make_entry<Radices<15, 8, 8, 16>, 1024, 1, OPT_NT>(1024, 15),
        make_entry<Radices<9, 16, 16>, 128, 2, OPT_SEQ_TWIDDLE | OPT_PAIRED_IO | OPT_NT>(256, 9),
        make_entry<Radices<5, 4, 4>, 16, 8, OPT_PAIRED_IO | OPT_NT>(16, 5),
        // each pass-0 row of the next group requested right after its DFT (measured: 6-8 % off
        // the forward here; no gain for (1024, 15) or (256, 9), whose variants were dropped)
        make_entry<Radices<15, 16, 8>, 64, 2, OPT_SEQ_TWIDDLE | OPT_PAIRED_IO | OPT_NT | OPT_EARLY_FETCH>(128, 15),
    };
    v.insert(v.end(), e, e + sizeof(e) / sizeof(e[0]));
}
} // namespace bt

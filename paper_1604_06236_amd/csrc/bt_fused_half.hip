// Uniform batches of K = 1024 blocks with the half-block LDS exchange body of bt_half.hpp (the
// transform of eq. (6) with the radix plan [M, 32, 32]): one block at a time per 512-thread
// workgroup, N/2 points of LDS (60 KB for M = 15 instead of 120 KB) and at most 128 VGPRs, so two
// workgroups share a CU.  Registered as extra schedules of the (1024, M) shapes for the
// autotuner; the tap-gradient launches of these entries run the uniform kernel of the same
// radix plan (the same base-root table), whose shared-tap reduction the half body lacks.
#include <vector>

#include "bt_api_internal.hpp"
#include "bt_half.hpp"

namespace bt {

constexpr int HALF_TB = 512;

// TAP_NT: per-block taps, streamed; shared taps (one filter for every block) stay cached
template <int M, int SIDE, bool TAP_NT>
__global__ void __launch_bounds__(HALF_TB, 4) half_lds_kernel(FusedArgs a)
{
    constexpr int N = 1024 * M;
    constexpr uint32_t CB = 8, FB = 4;
    __shared__ __attribute__((aligned(16))) c32 L[N / 2];
    poison_lds(L, N / 2);
    bool zero_tap = false;
    // base roots from the table of the plan [M, 32, 32]: pass 1's M entries, then pass 2's 32 M
    HalfThread<M> h;
    h.init(threadIdx.x, a.tw, 1, a.tw + M);
    for (int64_t b = blockIdx.x; b < a.nblocks; b += gridDim.x) {
        const rsrc_t ri = make_rsrc(a.in + b * N, N * CB), ro = make_rsrc(a.out + b * N, N * CB);
        const rsrc_t rt = make_rsrc(a.taps + (TAP_NT ? b * N : 0), N * FB);
        half_block<M, SIDE, TAP_NT>(h, L, ri, ro, rt, ro, ro, a.div, true, zero_tap);
    }
    if (zero_tap && a.div && a.status) *a.status = 1;
}

template <int M, int SIDE>
hipError_t half_launch(const FusedArgs &a, unsigned grid, hipStream_t s)
{
    if (a.tap_stride == 0)
        hipLaunchKernelGGL((half_lds_kernel<M, SIDE, false>), dim3(grid), dim3(HALF_TB), 0, s, a);
    else
        hipLaunchKernelGGL((half_lds_kernel<M, SIDE, true>), dim3(grid), dim3(HALF_TB), 0, s, a);
    return hipGetLastError();
}

// the tap-gradient launches reuse the uniform kernel instances of the shape's other schedules
// ([15, 32, 32] non-temporal for M = 15, the default plan otherwise)
template <int M>
FusedEntry half_entry()
{
    constexpr int OPT_TG = M == 15 ? OPT_NT : 0;
    FusedEntry e = make_entry<Radices<M, 32, 32>, HALF_TB, 1, OPT_TG>(1024, M);
    e.opt |= OPT_HALF_LDS | OPT_NT;
    e.lds_bytes = (1024 * M / 2) * int(sizeof(c32));
    e.launch[0][0] = &half_launch<M, SIDE_IN>;
    e.launch[1][0] = &half_launch<M, SIDE_OUT>;
    // occupancy (two workgroups per CU) is the same for both tap policies
    e.kernel[0][0] = reinterpret_cast<const void *>(&half_lds_kernel<M, SIDE_IN, false>);
    e.kernel[1][0] = reinterpret_cast<const void *>(&half_lds_kernel<M, SIDE_OUT, false>);
    return e;
}

void register_fused_half(std::vector<FusedEntry> &v)
{
    const FusedEntry e[] = {half_entry<3>(), half_entry<5>(), half_entry<7>(), half_entry<9>(),
                            half_entry<15>()};
    v.insert(v.end(), e, e + sizeof(e) / sizeof(e[0]));
}

} // namespace bt

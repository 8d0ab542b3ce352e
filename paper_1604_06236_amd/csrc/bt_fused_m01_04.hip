// Default fused schedules for M = 1..4 and every supported K (1..1024).
#include <vector>
#include "bt_fused.hpp"

#define BT_ALL_K(M) \
    default_entry<1, M>(), default_entry<2, M>(), default_entry<4, M>(), default_entry<8, M>(), \
    default_entry<16, M>(), default_entry<32, M>(), default_entry<64, M>(), default_entry<128, M>(), \
    default_entry<256, M>(), default_entry<512, M>(), default_entry<1024, M>()

namespace bt {
void register_fused_m01_04(std::vector<FusedEntry> &v)
{
    const FusedEntry e[] = {BT_ALL_K(1),BT_ALL_K(2),BT_ALL_K(3),BT_ALL_K(4)};
    v.insert(v.end(), e, e + sizeof(e) / sizeof(e[0]));
}
} // namespace bt

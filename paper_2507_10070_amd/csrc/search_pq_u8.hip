// search_pq_u8.hip -- the compressed-navigation (NAV_PQ) batch search and
// server kernels for uint8 vectors, in a unit of their own so that the kernel
// sets of the three element types compile in parallel.
#define FA_SEARCH_TEMPLATES_ONLY
#include "search_kernel.hip"

namespace fa {

hipError_t launch_search_pq_u8(const SearchArgs &a, int transport, int wpb, bool pers,
                              hipStream_t st) {
  return launch_c<DT_U8, NAV_PQ>(a, a.nav_stride / 128, transport, wpb, pers, st);
}

hipError_t launch_server_pq_u8(const ServerArgs &a, int wpb, int64_t *res, hipStream_t st) {
  return launch_server_c<DT_U8, NAV_PQ>(a, wpb, res, st);
}

}  // namespace fa

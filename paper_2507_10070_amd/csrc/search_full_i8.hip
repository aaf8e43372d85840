// search_full_i8.hip -- the full-precision-navigation (NAV_FULL) batch search
// and server kernels for int8 vectors, in a unit of their own so that the
// kernel sets compile in parallel.
#define FA_SEARCH_TEMPLATES_ONLY
#include "search_kernel.hip"

namespace fa {

hipError_t launch_search_full_i8(const SearchArgs &a, int transport, int wpb, bool pers,
                                hipStream_t st) {
  return launch_c<DT_I8, NAV_FULL>(a, a.nav_stride / 128, transport, wpb, pers, st);
}

hipError_t launch_server_full_i8(const ServerArgs &a, int wpb, int64_t *res, hipStream_t st) {
  return launch_server_c<DT_I8, NAV_FULL>(a, wpb, res, st);
}

}  // namespace fa

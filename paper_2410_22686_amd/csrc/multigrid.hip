// Complex-shifted geometric multigrid for Step 2 with a variable coefficient
// (one V-cycle per frequency slice).
#include "common.hpp"
#include "launch.hpp"

namespace pcop {

bool launch_mg_solve(const Geo& g, void* spec, bool fp32, const PrecondTables& tb, hipStream_t st) {
  (void)g; (void)spec; (void)fp32; (void)tb; (void)st;
  return false;
}

}  // namespace pcop

// Forward in-place time pass, FP32 complex data.
#include "time_ip.hpp"

namespace pcop {

template void launch_time_ip_dir<float, true>(int, const Geo&, const double*, cx<float>*, double*,
                                                     const PrecondTables&, const cx<float>*, const double*, int, int,
                                                     hipStream_t);

}  // namespace pcop

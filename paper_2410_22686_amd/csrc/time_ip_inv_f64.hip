// Inverse in-place time pass, FP64 complex data.
#include "time_ip.hpp"

namespace pcop {

template void launch_time_ip_dir<double, false>(int, const Geo&, const double*, cx<double>*, double*,
                                                     const PrecondTables&, const cx<double>*, const double*, int, int,
                                                     hipStream_t);

}  // namespace pcop

// sans_sur.hip -- surrogate-mode kernels of the models that have a network
// (the parallelepiped and the ellipsoid of revolution).
#include "sans_kernels.hpp"

namespace sans {

SurFn sur_kernel(int kind)
{
    if (kind == kParallelepiped) return k_trace_sur<kParallelepiped>;
    if (kind == kEllipsoid) return k_trace_sur<kEllipsoid>;
    return nullptr;
}

QueueFn sur_queue_kernel(int kind)
{
    if (kind == kParallelepiped) return k_trace_queue<kParallelepiped>;
    if (kind == kEllipsoid) return k_trace_queue<kEllipsoid>;
    return nullptr;
}

DatasetFn dataset_kernel(int kind)
{
    if (kind == kParallelepiped) return k_pq_dataset<kParallelepiped>;
    if (kind == kEllipsoid) return k_pq_dataset<kEllipsoid>;
    return nullptr;
}

}  // namespace sans

// Single-precision instantiation of the step kernels.
#define SS_DISPATCH_IMPL
#include "ss_dispatch.hpp"
namespace ss {
SS_INSTANTIATE(float)
}

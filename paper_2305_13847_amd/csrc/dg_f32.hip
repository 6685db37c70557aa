// FP32-bulk instantiation of the kernels and launchers (the split and the
// state reconstruction stay FP64 inside the kernels).
#include "dg_launch.h"
namespace dgm {
template struct Launch<float>;
}

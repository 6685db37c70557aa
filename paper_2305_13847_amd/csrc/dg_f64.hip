// FP64 instantiation of the kernels and launchers.
#include "dg_launch.h"
namespace dgm {
template struct Launch<double>;
}

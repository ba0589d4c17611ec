// Stage kernels of the 3D order-3 element in FP64.
#include "gb_launch.hpp"
GB_DEFINE_SHAPE(3, 3, f64, double)

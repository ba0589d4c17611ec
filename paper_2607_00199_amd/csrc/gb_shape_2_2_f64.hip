// Stage kernels of the 2D order-2 element in FP64.
#include "gb_launch.hpp"
GB_DEFINE_SHAPE(2, 2, f64, double)

// Stage kernels of the 2D order-5 element in FP64.
#include "gb_launch.hpp"
GB_DEFINE_SHAPE(2, 5, f64, double)

// Stage kernels of the 3D order-2 element in FP32.
#include "gb_launch.hpp"
GB_DEFINE_SHAPE(3, 2, f32, float)

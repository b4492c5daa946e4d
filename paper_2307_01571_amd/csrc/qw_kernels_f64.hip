// FP64 instantiation of the split-operator kernels.
#include "qw_kernels.inl"
QW_DEFINE_LAUNCHERS(double, f64)

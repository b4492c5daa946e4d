// FP32 instantiation of the split-operator kernels (float state and
// butterflies; phases and reductions in double, see qw_kernels.inl).
#include "qw_kernels.inl"
QW_DEFINE_LAUNCHERS(float, f32)

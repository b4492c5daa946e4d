// FP32 instantiation of the batched split-operator kernels.  Built with
// machine loop-invariant code motion off: in the persistent item loop it
// would hoist the constants of the in-kernel sin/cos out of the loop and
// hold them in registers for the whole kernel.
#define QW_BATCH_VARIANTS QW_BATCH_VARIANTS_float
#include "qw_batch.inl"
QW_DEFINE_BATCH_LAUNCHERS(float, f32)

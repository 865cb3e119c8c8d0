// One 16-bit operand form of the statistics kernels: __bf16, hi only (accuracy control).
#define FV_FORM_T __bf16
#define FV_FORM_SPLIT 0
#define FV_FORM_COMP 0
#define FV_FORM_NAME(x) x##_bf16
#include "fv_kernels16.inc"

// One 16-bit operand form of the statistics kernels: __bf16, three-product hi/lo split.
#define FV_FORM_T __bf16
#define FV_FORM_SPLIT 1
#define FV_FORM_COMP 0
#define FV_FORM_NAME(x) x##_bf16s
#include "fv_kernels16.inc"

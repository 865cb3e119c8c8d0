// One 16-bit operand form of the statistics kernels: _Float16, three-product hi/lo split.
#define FV_FORM_T _Float16
#define FV_FORM_SPLIT 1
#define FV_FORM_COMP 0
#define FV_FORM_NAME(x) x##_f16s
#include "fv_kernels16.inc"

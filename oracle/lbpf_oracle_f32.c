/*
 * lbpf_oracle_f32.c -- the LB oracle's algorithm in single precision.
 *
 * TEST INFRASTRUCTURE ONLY.  This translation unit compiles lbpf_oracle.c
 * unchanged with every `double` read as `float` (and, through the build
 * flags, every floating constant in single precision).  The system headers
 * are included first, so the math library keeps its double prototypes: a
 * sqrt is computed in double and rounded once to float where it is stored.
 * The result is the same step, rounded as an FP32 implementation of it
 * would be, and serves as evidence of what FP32 state and arithmetic alone
 * cost the method over n steps.  It is never the reference of a parity test.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define double float
#include "lbpf_oracle.c"

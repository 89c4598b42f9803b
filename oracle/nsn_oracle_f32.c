/*
 * The oracle's source evaluated in single precision -- TEST INFRASTRUCTURE ONLY.
 *
 * Every double of nsn_oracle.c (its API included) becomes a float; the system
 * headers are included first so that the substitution stays out of them.  Not an
 * oracle: the per-row parity tests use the distance between this build and the FP64
 * build, on the same inputs, as an estimate of what FP32 rounding alone does to each
 * quantity of a Newton iteration (cancellation included).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#define double float
#include "nsn_oracle.c"

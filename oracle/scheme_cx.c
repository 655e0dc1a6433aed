/*
 * The oracle's step with complex state (test infrastructure only): the same
 * source as scheme.c compiled with C99 double complex as the state scalar,
 * for complex-step directional derivatives of the step (see sreal.h).
 */
#define RGO_COMPLEX 1
#include "scheme.c"

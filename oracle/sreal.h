/*
 * The scalar type of the state-dependent arithmetic of the oracle's step
 * (test infrastructure only).  scheme.c is compiled twice:
 *   - as itself: sreal is double, and this is the oracle proper;
 *   - through scheme_cx.c with RGO_COMPLEX defined: sreal is C99 double
 *     complex, and the step gives the complex-step directional derivative:
 *     with state U + i h d (h about 1e-30) the imaginary part of the
 *     result divided by h is the derivative of the step along d, exact to
 *     rounding (no subtractive cancellation).
 * Geometry stays real in both.  Every branch of the step (MinMod, the HLL
 * branch and the Davis speeds' min/max, the multidimensional solver's
 * maxima, the clamps of the fast speed's discriminant and of the
 * flattener) decides on real parts, so the complex build differentiates
 * the branch the real step takes.  |x| continues analytically as
 * x sign(Re x).
 */
#ifndef RGO_SREAL_H
#define RGO_SREAL_H

#include <math.h>

#ifdef RGO_COMPLEX
#include <complex.h>
typedef double complex sreal;
static inline double SRE(sreal x) { return creal(x); }
static inline sreal s_sqrt(sreal x) { return csqrt(x); }
static inline sreal s_abs(sreal x) { return creal(x) < 0.0 ? -x : x; }
/* fmin / fmax by real part; the first argument on ties */
static inline sreal s_min(sreal a, sreal b) { return creal(b) < creal(a) ? b : a; }
static inline sreal s_max(sreal a, sreal b) { return creal(b) > creal(a) ? b : a; }
#else
typedef double sreal;
#define SRE(x) (x)
#define s_sqrt sqrt
#define s_abs fabs
#define s_min fmin
#define s_max fmax
#endif

#endif

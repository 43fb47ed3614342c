/*
 * CPU oracle for the loop hafnian and its subset terms -- TEST INFRASTRUCTURE.
 *
 * A plain, slow, obviously-correct reference written from the paper (Quesada
 * et al., "Quadratic speedup for simulating Gaussian boson sampling"), used only
 * by the test-suite, the smoke check and the CPU-baseline leg of the benchmark.
 * It shares no source with the HIP library and must never be linked into it.
 *
 * Every routine exists twice: suffix _d computes in double, suffix _ld in
 * x87 long double (the precision the paper's Sec. IV uses for its accuracy and
 * timing figures).  Inputs are row-major interleaved (re, im) doubles.
 * The arithmetic itself lives in lhaf_body.h.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_DP_MAX_N 26
#define ORACLE_PT_MAX_N 64
#define ORACLE_CHUNK 4096ULL

/* ---- double instantiation ---- */
#define SFX(name) name##_d
#define REAL double
#define CPLX double complex
#define RSQRT(x) sqrt(x)
#define RABS(x) fabs(x)
#define ZABS(z) cabs(z)
#define ZCONJ(z) conj(z)
#define ZRE(z) creal(z)
#define ZIM(z) cimag(z)
#include "lhaf_body.h"
#undef SFX
#undef REAL
#undef CPLX
#undef RSQRT
#undef RABS
#undef ZABS
#undef ZCONJ
#undef ZRE
#undef ZIM

/* ---- long double instantiation ---- */
#define SFX(name) name##_ld
#define REAL long double
#define CPLX long double complex
#define RSQRT(x) sqrtl(x)
#define RABS(x) fabsl(x)
#define ZABS(z) cabsl(z)
#define ZCONJ(z) conjl(z)
#define ZRE(z) creall(z)
#define ZIM(z) cimagl(z)
#include "lhaf_body.h"

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

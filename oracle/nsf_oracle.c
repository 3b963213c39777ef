/*
 * CPU oracle for the compressible Navier-Stokes residual and the
 * three-stage low-storage Runge-Kutta update of Jammy, Jacobs & Sandham
 * (arXiv 1610.09146), written in plain C.
 *
 * TEST INFRASTRUCTURE ONLY: it exists to check the GPU library. Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, headers or constants with the GPU path.
 *
 * The arithmetic lives in nsf_oracle_body.inc, instantiated here for
 * double (symbols *_d) and for x87 extended long double (symbols *_ld); the
 * long-double build supplies the round-off floor the double results are
 * judged against. Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC.
 *
 * Pins (checked by the CPU tests, not by comparison with the GPU):
 * closed-form modified wavenumbers of the first, second and cross
 * derivatives; exact initial kinetic energy, enstrophy, extrema and
 * energy-residual mean of the Taylor-Green state; the initial kinetic-energy
 * decay rate; fourth-order convergence of every residual field to the exact
 * residual of the continuous equations (symbolic, divergence form); the exact
 * discrete residual of one-dimensional compressive waves (trigonometric
 * polynomials through the modified wavenumbers), which fixes the skew split
 * and the pressure work of the energy equation; discrete conservation of
 * mass and momentum; third-order time accuracy; dense Kronecker-operator
 * brute force on small grids. Copies with a planted mistake in any of these
 * terms fail at least one pin.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PI_LD 3.141592653589793238462643383279502884L

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the n-th output (n >= 1) of
 * the stream whose state starts at `seed` is mix(seed + n * 0x9e3779b97f4a7c15).
 * Counter-based use: output number counter+1. The 53 high bits give a
 * uniform double in [0, 1). */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double oracle_splitmix_uniform(uint64_t seed, uint64_t counter)
{
    return (double)(oracle_splitmix64(seed, counter) >> 11) * 0x1.0p-53;
}

#ifdef _OPENMP
#include <omp.h>
void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int oracle_get_threads(void) { return omp_get_max_threads(); }
#else
void oracle_set_threads(int n) { (void)n; }
int oracle_get_threads(void) { return 1; }
#endif

#define REAL double
#define SFX _d
#define SIN sin
#define COS cos
#include "nsf_oracle_body.inc"
#undef REAL
#undef SFX
#undef SIN
#undef COS

#define REAL long double
#define SFX _ld
#define SIN sinl
#define COS cosl
#include "nsf_oracle_body.inc"
#undef REAL
#undef SFX
#undef SIN
#undef COS

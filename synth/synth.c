/*
 * Seeded synthetic inputs shared by the oracle side and the GPU side.
 *
 * This file holds random-number generation only, none of the transform,
 * Poisson or power-spectrum arithmetic.  Every value is a pure function of
 * (seed, stream, counter), so any element can be regenerated on its own.
 *
 * Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014; the public-domain reference is Vigna's
 * splitmix64.c).  The state advances by the golden-ratio increment
 * 0x9e3779b97f4a7c15 and each output is the state passed through the
 * variant-13 finaliser.  Counter-based use: output i of a stream is the
 * finaliser applied to  state0 + (i + 1) * increment, where
 * state0 = finaliser(seed + (stream + 1) * increment).
 *
 * Derived variates:
 *   uniform(i)  = (u64(i) >> 11) * 2^-53                    in [0, 1)
 *   normal(i)   = sqrt(-2 ln u1) * cos(2 pi u2)             Box-Muller,
 *                 u1 = ((u64(2i) >> 11) + 1) * 2^-53 in (0, 1],
 *                 u2 = (u64(2i+1) >> 11) * 2^-53,
 *                 evaluated in double precision.
 *   normal_f32  = normal rounded to float (round to nearest even).
 */
#include <math.h>
#include <stdint.h>

#define SM64_GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t sm64_state0(uint64_t seed, uint64_t stream)
{
    return sm64_mix(seed + (stream + 1) * SM64_GAMMA);
}

static inline uint64_t sm64_at(uint64_t s0, uint64_t i)
{
    return sm64_mix(s0 + (i + 1) * SM64_GAMMA);
}

static inline double u01_closed_open(uint64_t v) { return (double)(v >> 11) * 0x1.0p-53; }
static inline double u01_open_closed(uint64_t v) { return (double)((v >> 11) + 1) * 0x1.0p-53; }

static inline double normal_at(uint64_t s0, uint64_t i)
{
    const double two_pi = 6.283185307179586476925286766559;
    double u1 = u01_open_closed(sm64_at(s0, 2 * i));
    double u2 = u01_closed_open(sm64_at(s0, 2 * i + 1));
    return sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
}

/* Output i of a SplitMix64 generator whose state is `state` before the
 * first step (the raw generator, exposed for known-answer tests). */
uint64_t synth_sm64_raw(uint64_t state, uint64_t i)
{
    return sm64_at(state, i);
}

uint64_t synth_u64(uint64_t seed, uint64_t stream, uint64_t i)
{
    return sm64_at(sm64_state0(seed, stream), i);
}

void synth_uniform_f64(uint64_t seed, uint64_t stream, uint64_t offset, int64_t n, double *out)
{
    uint64_t s0 = sm64_state0(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = u01_closed_open(sm64_at(s0, offset + (uint64_t)i));
}

void synth_normal_f64(uint64_t seed, uint64_t stream, uint64_t offset, int64_t n, double *out)
{
    uint64_t s0 = sm64_state0(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = normal_at(s0, offset + (uint64_t)i);
}

void synth_normal_f32(uint64_t seed, uint64_t stream, uint64_t offset, int64_t n, float *out)
{
    uint64_t s0 = sm64_state0(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = (float)normal_at(s0, offset + (uint64_t)i);
}

/* Integer draws in [0, m) by the multiply-shift map of the top 32 bits
 * (used for lattice-size and arrival choices, never for field values). */
void synth_choice(uint64_t seed, uint64_t stream, int64_t n, int64_t m, int64_t *out)
{
    uint64_t s0 = sm64_state0(seed, stream);
    for (int64_t i = 0; i < n; ++i)
        out[i] = (int64_t)(((sm64_at(s0, (uint64_t)i) >> 32) * (uint64_t)m) >> 32);
}

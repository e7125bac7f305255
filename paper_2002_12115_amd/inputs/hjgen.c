/*
 * hjgen.c -- seeded synthetic inputs for the 19-point Jacobi pressure sweep.
 *
 * This module only draws numbers. It holds none of the sweep's arithmetic and
 * is shared, as plain host arrays, by the CPU oracle and by the HIP path.
 *
 * Generator: a counter-based SplitMix64 stream (Steele, Lea, Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014). Value number n of
 * a stream whose state starts at s is mix(s + (n+1)*GAMMA), where mix is the
 * published SplitMix64 finalizer and GAMMA = 0x9e3779b97f4a7c15. A field's
 * stream starts at s = mix(seed) ^ (field_id << 56), so every (seed, field,
 * cell) triple has its own value and the result does not depend on the order
 * or thread count used to fill an array.
 *
 * Uniforms use the top 53 bits: u = (x >> 11) * 2^-53, in [0, 1).
 * Normals use Box and Muller (1958) on the counter pair (2m, 2m+1):
 *   r = sqrt(-2 ln(1 - u0)), z(2m) = r cos(2 pi u1), z(2m+1) = r sin(2 pi u1).
 *
 * Field ids (dense C order [nx][ny][nz], k fastest, linear index = cell):
 *   0 p ~ U[0,1)          1..3 a0..a2 ~ U[0.9,1.1)    5..7 b0..b2 ~ U[-0.05,0.05)
 *   8..10 c0..c2 ~ U[0.9,1.1)    12 wrk1 ~ N(0, sigma)
 *   4 a3 = 1 / (a0+a1+a2 + c0+c1+c2 + 4(|b0|+|b1|+|b2|) + 0.1), from the drawn values
 *   11 bnd = 1 on the interior, 0 on the one-cell shell (or a random 0/1 interior mask)
 *   13 batch instance sizes (index 3*inst + axis)
 * The recipe (distributions and the a3 rule) is the workload definition of the
 * Himeno-style pressure solve used to exercise the Jacobi sweep; the paper
 * names that workload (section 5.1.1) but prints no formula or sizes.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define HJGEN_GAMMA 0x9e3779b97f4a7c15ULL

uint64_t hjgen_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_state(uint64_t seed, int field)
{
    return hjgen_mix(seed) ^ ((uint64_t)(unsigned)field << 56);
}

static inline uint64_t stream_value(uint64_t state, uint64_t n)
{
    return hjgen_mix(state + (n + 1) * HJGEN_GAMMA);
}

static inline double to_unit(uint64_t x)
{
    return (double)(x >> 11) * 0x1.0p-53;
}

uint64_t hjgen_bits(uint64_t seed, int field, uint64_t n)
{
    return stream_value(stream_state(seed, field), n);
}

double hjgen_uniform(uint64_t seed, int field, uint64_t n)
{
    return to_unit(hjgen_bits(seed, field, n));
}

static inline double normal_at(uint64_t state, uint64_t n, double sigma)
{
    const uint64_t m = n >> 1;
    const double u0 = to_unit(stream_value(state, 2 * m));
    const double u1 = to_unit(stream_value(state, 2 * m + 1));
    const double r = sqrt(-2.0 * log(1.0 - u0));
    const double t = 6.283185307179586476925286766559 * u1;
    return sigma * ((n & 1) ? r * sin(t) : r * cos(t));
}

double hjgen_normal(uint64_t seed, int field, uint64_t n, double sigma)
{
    return normal_at(stream_state(seed, field), n, sigma);
}

static inline double draw(uint64_t seed, int field, uint64_t n)
{
    const double u = hjgen_uniform(seed, field, n);
    if (field == 0) return u;
    if (field >= 5 && field <= 7) return -0.05 + 0.1 * u;
    return 0.9 + 0.2 * u; /* a0..a2, c0..c2 */
}

/* Value of field `field` at dense cell n = (i*ny + j)*nz + k.
 * bnd_mode 0: interior 1, shell 0.  bnd_mode 1: interior Bernoulli(1/2) mask
 * drawn from stream 11, shell 0. */
static inline double field_value(uint64_t seed, int field, int nx, int ny, int nz,
                                 uint64_t n, double sigma, int bnd_mode)
{
    switch (field) {
    case 4: {
        double sa = draw(seed, 1, n) + draw(seed, 2, n) + draw(seed, 3, n);
        double sc = draw(seed, 8, n) + draw(seed, 9, n) + draw(seed, 10, n);
        double sb = fabs(draw(seed, 5, n)) + fabs(draw(seed, 6, n)) + fabs(draw(seed, 7, n));
        return 1.0 / (sa + sc + 4.0 * sb + 0.1);
    }
    case 11: {
        const uint64_t plane = (uint64_t)ny * (uint64_t)nz;
        const int i = (int)(n / plane);
        const int j = (int)((n / (uint64_t)nz) % (uint64_t)ny);
        const int k = (int)(n % (uint64_t)nz);
        if (i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1) return 0.0;
        if (bnd_mode == 0) return 1.0;
        return (hjgen_bits(seed, 11, n) >> 63) ? 1.0 : 0.0;
    }
    case 12:
        return hjgen_normal(seed, 12, n, sigma);
    default:
        return draw(seed, field, n);
    }
}

/* Fill a dense [nx][ny][nz] array with field `field` (0..12).
 * Returns 0, or -1 for a bad field id or shape. */
int hjgen_fill_f64(uint64_t seed, int field, int nx, int ny, int nz,
                   double sigma, int bnd_mode, double* out)
{
    if (field < 0 || field > 12 || nx < 1 || ny < 1 || nz < 1 || !out) return -1;
    const long long total = (long long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < total; ++n)
        out[n] = field_value(seed, field, nx, ny, nz, (uint64_t)n, sigma, bnd_mode);
    return 0;
}

/* Same values rounded to float (round to nearest even, the C conversion rule
 * under the default rounding mode). */
int hjgen_fill_f32(uint64_t seed, int field, int nx, int ny, int nz,
                   double sigma, int bnd_mode, float* out)
{
    if (field < 0 || field > 12 || nx < 1 || ny < 1 || nz < 1 || !out) return -1;
    const long long total = (long long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < total; ++n)
        out[n] = (float)field_value(seed, field, nx, ny, nz, (uint64_t)n, sigma, bnd_mode);
    return 0;
}

/* Instance seeds and sizes for a batch of independent solves.
 * Instance seed: mix(seed ^ (inst+1)).  Sizes from stream 13 of `seed`,
 * index 3*inst + axis: nx, ny ~ U{lo_xy..hi_xy}, nz ~ U{lo_z..hi_z}. */
int hjgen_batch(uint64_t seed, int n_inst, int lo_xy, int hi_xy, int lo_z, int hi_z,
                int* nx, int* ny, int* nz, uint64_t* inst_seed)
{
    if (n_inst < 0 || hi_xy < lo_xy || hi_z < lo_z) return -1;
    for (int t = 0; t < n_inst; ++t) {
        const int lo[3] = {lo_xy, lo_xy, lo_z};
        const int hi[3] = {hi_xy, hi_xy, hi_z};
        int d[3];
        for (int a = 0; a < 3; ++a) {
            const double u = hjgen_uniform(seed, 13, (uint64_t)(3 * t + a));
            int v = lo[a] + (int)floor(u * (double)(hi[a] - lo[a] + 1));
            if (v > hi[a]) v = hi[a];
            d[a] = v;
        }
        if (nx) nx[t] = d[0];
        if (ny) ny[t] = d[1];
        if (nz) nz[t] = d[2];
        if (inst_seed) inst_seed[t] = hjgen_mix(seed ^ (uint64_t)(t + 1));
    }
    return 0;
}

/* Values of field `field` at selected dense linear indices of an
 * [nx][ny][nz] grid (any order, any count): the same numbers hjgen_fill_f64
 * puts at those positions. */
int hjgen_values_f64(uint64_t seed, int field, int nx, int ny, int nz, double sigma,
                     int bnd_mode, long long count, const long long* idx, double* out)
{
    if (field < 0 || field > 12 || nx < 1 || ny < 1 || nz < 1 || !idx || !out) return -1;
    const long long total = (long long)nx * ny * nz;
    for (long long q = 0; q < count; ++q)
        if (idx[q] < 0 || idx[q] >= total) return -1;
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < count; ++q)
        out[q] = field_value(seed, field, nx, ny, nz, (uint64_t)idx[q], sigma, bnd_mode);
    return 0;
}

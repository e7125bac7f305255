// sanitize_driver.cpp -- exercises the host-side C/C++ of the project (the
// input generator, the CPU oracle, the genetic search engine) under
// AddressSanitizer and UndefinedBehaviorSanitizer. Built and run by
// tests/test_sanitize.py; any sanitizer report aborts with a non-zero status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hj_ga.hpp"

extern "C" {
// inputs/hjgen.c
uint64_t hjgen_mix(uint64_t z);
uint64_t hjgen_bits(uint64_t seed, int field, uint64_t n);
double hjgen_uniform(uint64_t seed, int field, uint64_t n);
double hjgen_normal(uint64_t seed, int field, uint64_t n, double sigma);
int hjgen_fill_f64(uint64_t seed, int field, int nx, int ny, int nz, double sigma, int bnd_mode, double* out);
int hjgen_fill_f32(uint64_t seed, int field, int nx, int ny, int nz, double sigma, int bnd_mode, float* out);
int hjgen_batch(uint64_t seed, int n_inst, int lo_xy, int hi_xy, int lo_z, int hi_z, int* nx, int* ny, int* nz,
                uint64_t* seeds);
int hjgen_values_f64(uint64_t seed, int field, int nx, int ny, int nz, double sigma, int bnd_mode,
                     long long n, const long long* idx, double* out);
// oracle/oracle.c
int oracle_sweep(int nx, int ny, int nz, double* const f[14], int n_iter, double omega, double* gosa_hist,
                 int nthreads);
double oracle_residual(int nx, int ny, int nz, double* const f[14], int nthreads);
int oracle_cells(int nx, int ny, int nz, double* const f[14], double omega, long long n_cells,
                 const long long* idx, double* ss_out, double* wrk2_out);
}

static int failures = 0;

static void expect(bool ok, const char* what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static void generator_and_oracle(int nx, int ny, int nz, int bnd_mode)
{
    const size_t n = (size_t)nx * ny * nz;
    std::vector<std::vector<double>> f(14, std::vector<double>(n));
    std::vector<float> f32(n);
    for (int q = 0; q < 13; ++q) {
        expect(hjgen_fill_f64(2002, q, nx, ny, nz, 0.01, bnd_mode, f[q].data()) == 0, "fill_f64");
        expect(hjgen_fill_f32(2002, q, nx, ny, nz, 0.01, bnd_mode, f32.data()) == 0, "fill_f32");
    }
    f[13] = f[0];
    std::vector<long long> idx;
    for (size_t c = 0; c < n; c += 7) idx.push_back((long long)c);
    std::vector<double> vals(idx.size());
    expect(hjgen_values_f64(2002, 0, nx, ny, nz, 0.01, bnd_mode, (long long)idx.size(), idx.data(),
                            vals.data()) == 0, "values_f64");
    for (size_t q = 0; q < idx.size(); ++q) expect(vals[q] == f[0][(size_t)idx[q]], "values equal fill");

    double* ptr[14];
    for (int q = 0; q < 14; ++q) ptr[q] = f[q].data();
    for (int threads : {1, 3}) {
        std::vector<std::vector<double>> g = f;
        double* gp[14];
        for (int q = 0; q < 14; ++q) gp[q] = g[q].data();
        std::vector<double> hist(4);
        expect(oracle_sweep(nx, ny, nz, gp, 4, 0.8, hist.data(), threads) == 0, "oracle_sweep");
        expect(oracle_sweep(nx, ny, nz, gp, 0, 0.8, nullptr, threads) == 0, "oracle_sweep zero");
        expect(oracle_residual(nx, ny, nz, gp, threads) >= 0.0, "oracle_residual");
    }
    // one iteration at the interior cells, and an index on the shell (-5)
    std::vector<long long> cells;
    for (int i = 1; i < nx - 1; i += 2)
        for (int j = 1; j < ny - 1; j += 3)
            for (int k = 1; k < nz - 1; k += 2) cells.push_back(((long long)i * ny + j) * nz + k);
    std::vector<double> ss(cells.size()), w2(cells.size());
    expect(oracle_cells(nx, ny, nz, ptr, 0.8, (long long)cells.size(), cells.data(), ss.data(), w2.data()) == 0,
           "oracle_cells");
    const long long shell = 0;
    expect(oracle_cells(nx, ny, nz, ptr, 0.8, 1, &shell, ss.data(), w2.data()) == -5, "oracle_cells shell");
}

static void error_paths()
{
    double x = 0;
    double* ptr[14];
    for (int q = 0; q < 14; ++q) ptr[q] = &x;
    ptr[5] = nullptr;
    expect(oracle_sweep(3, 3, 3, ptr, 1, 0.8, nullptr, 1) == -1, "null array");
    ptr[5] = &x;
    expect(oracle_sweep(2, 3, 3, ptr, 1, 0.8, nullptr, 1) == -2, "shape");
    expect(oracle_sweep(3, 3, 3, ptr, -1, 0.8, nullptr, 1) == -3, "n_iter");
    expect(oracle_residual(3, 2, 3, ptr, 1) < 0.0, "residual shape");
    expect(hjgen_fill_f64(1, 13, 3, 3, 3, 0.01, 0, &x) != 0, "field id");
    int a[4], b[4], c[4];
    uint64_t s[4];
    expect(hjgen_batch(2002, 4, 17, 129, 33, 257, a, b, c, s) == 0, "batch");
    expect(hjgen_batch(2002, 4, 9, 3, 33, 257, a, b, c, s) != 0, "batch range");
    (void)hjgen_mix(~0ULL);
    (void)hjgen_bits(~0ULL, 12, ~0ULL);
    expect(std::isfinite(hjgen_normal(7, 12, 0, 0.01)), "normal");
    expect(hjgen_uniform(7, 1, 5) >= 0.0 && hjgen_uniform(7, 1, 5) < 1.0, "uniform");
}

static void genetic_search()
{
    struct Case { int L, M, T; double pc, pm; };
    const Case cases[] = {{6, 5, 4, 0.9, 0.05}, {11, 10, 10, 0.9, 0.05}, {1, 1, 1, 0.9, 0.05},
                          {20, 3, 2, 1.0, 1.0}, {8, 7, 3, 0.0, 0.0},    {5, 9, 6, 0.5, 0.5}};
    for (const Case& k : cases) {
        // some genes fail (NaN, negative, infinite): they count as 1000 s
        auto t = [&](uint32_t g) -> double {
            if (g % 7 == 3) return NAN;
            if (g % 11 == 5) return -1.0;
            if (g % 13 == 6) return INFINITY;
            return 1.0 + (double)__builtin_popcount(g ^ 0x2a5u);
        };
        const hjga::Result r = hjga::run(k.L, k.M, k.T, 2002, k.pc, k.pm, t);
        expect(r.history.size() == (size_t)k.M * k.T, "history size");
        expect(r.evaluations >= 1 && r.evaluations <= k.M * k.T, "evaluations");
        expect(r.best_time > 0.0 && r.best_time <= hjga::kFailTime, "best time");
        for (uint32_t g : r.history) expect(g < (1u << k.L), "gene within L bits");
    }
    const hjga::Result all_fail = hjga::run(6, 4, 3, 1, 0.9, 0.05, [](uint32_t) { return NAN; });
    expect(all_fail.best_time == hjga::kFailTime, "every gene failing scores 1000 s");
}

int main()
{
    for (int bnd_mode : {0, 1}) {
        generator_and_oracle(3, 3, 3, bnd_mode);
        generator_and_oracle(4, 5, 3, bnd_mode);
        generator_and_oracle(9, 7, 13, bnd_mode);
        generator_and_oracle(17, 20, 33, bnd_mode);
    }
    error_paths();
    genetic_search();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("sanitize ok\n");
    return 0;
}

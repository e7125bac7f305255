// hj_ga.cpp -- the genetic search engine (host code). The scheme and the
// choices this implementation fixes are described in hj_ga.hpp.
#include "hj_ga.hpp"

#include <cmath>
#include <map>

namespace hjga {

namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ULL;

uint64_t mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

}  // namespace

double uniform(uint64_t seed, uint64_t stream, uint64_t n)
{
    const uint64_t state = mix(seed + (stream + 1) * kGamma);
    return (double)(mix(state + (n + 1) * kGamma) >> 11) * 0x1.0p-53;
}

Result run(int L, int M, int T, uint64_t seed, double pc, double pm,
           const std::function<double(uint32_t)>& time_of)
{
    Result r;
    const uint32_t full = L >= 32 ? 0xffffffffu : ((1u << L) - 1u);
    std::vector<uint32_t> pop(M, 0u);
    for (int m = 0; m < M; ++m)
        for (int b = 0; b < L; ++b)
            if (uniform(seed, 0, (uint64_t)m * L + b) < 0.5) pop[m] |= 1u << b;

    std::map<uint32_t, double> measured;
    bool have_best = false;
    std::vector<double> fit(M);
    for (int g = 0; g < T; ++g) {
        r.history.insert(r.history.end(), pop.begin(), pop.end());
        int elite = 0;
        for (int m = 0; m < M; ++m) {
            auto it = measured.find(pop[m]);
            double t;
            if (it != measured.end()) {
                t = it->second;
            } else {
                t = time_of(pop[m]);
                if (!(t > 0.0) || !std::isfinite(t) || t > kFailTime) t = kFailTime;
                measured[pop[m]] = t;
                ++r.evaluations;
            }
            fit[m] = 1.0 / std::sqrt(t);
            if (fit[m] > fit[elite]) elite = m;
            if (!have_best || t < r.best_time) {
                r.best_time = t;
                r.best_gene = pop[m];
                have_best = true;
            }
        }
        if (g == T - 1) break;

        double total = 0.0;
        for (int m = 0; m < M; ++m) total += fit[m];
        auto roulette = [&](double u) {
            const double target = u * total;
            double acc = 0.0;
            for (int m = 0; m < M; ++m) {
                acc += fit[m];
                if (target < acc) return m;
            }
            return M - 1;
        };
        const uint64_t s_pick = 1 + 4 * (uint64_t)g, s_cross = s_pick + 1, s_point = s_pick + 2,
                       s_mut = s_pick + 3;
        std::vector<uint32_t> next;
        next.reserve(M);
        next.push_back(pop[elite]);
        uint64_t draw = 0, pair = 0, child = 0;
        while ((int)next.size() < M) {
            const uint32_t a = pop[roulette(uniform(seed, s_pick, draw++))];
            const uint32_t b = pop[roulette(uniform(seed, s_pick, draw++))];
            uint32_t c1 = a, c2 = b;
            if (L > 1 && uniform(seed, s_cross, pair) < pc) {
                const int point = 1 + (int)std::floor(uniform(seed, s_point, pair) * (double)(L - 1));
                const uint32_t low = (1u << point) - 1u;
                c1 = (a & low) | (b & ~low & full);
                c2 = (b & low) | (a & ~low & full);
            }
            ++pair;
            for (uint32_t c : {c1, c2}) {
                if ((int)next.size() >= M) break;
                for (int bit = 0; bit < L; ++bit)
                    if (uniform(seed, s_mut, child * L + bit) < pm) c ^= 1u << bit;
                ++child;
                next.push_back(c);
            }
        }
        pop.swap(next);
    }
    return r;
}

}  // namespace hjga

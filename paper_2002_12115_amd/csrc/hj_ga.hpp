// hj_ga.hpp -- the paper's genetic search, used as the autotuner's search
// strategy (internal).
//
// The paper finds the loops to offload with a genetic algorithm (sections 3.2
// and 4, parameters in section 5.1.2). One gene bit per decision. Every
// individual is built and timed, and its fitness is (time)^(-1/2). A
// measurement that fails or exceeds the time limit counts as 1000 s. Parents
// are chosen by roulette on fitness; the best individual is carried to the
// next generation unchanged (elitism). Crossover has probability Pc and
// mutation probability Pm per bit. After T generations the best individual
// measured is the answer.
// Here the decisions are the kernel's configuration bits instead of
// offload directives, and "build and time" is a timed sweep on the caller's
// arrays. Identical genes are measured once.
//
// Where the paper leaves a choice open, this implementation fixes it:
//  - crossover is one-point, at a point drawn uniformly from 1..L-1; the
//    low bits come from the first parent;
//  - parents are drawn in pairs, each pair giving two children (the last
//    child is dropped when the population is full);
//  - ties in fitness go to the lowest index, and ties in time to the first
//    individual measured.
// Random numbers come from a counter-based SplitMix64 (Steele, Lea, Flood
// 2014). Number n of stream s under seed q is the n-th output of the
// SplitMix64 sequence whose state starts at mix(q + (s+1)*GAMMA), reduced to
// [0,1) by its top 53 bits. Streams: 0 holds the initial bits (individual m,
// bit b at n = m*L + b). The step from generation g to g+1 uses stream
// 1+4g for roulette draws (sequential), 2+4g for the crossover decision of
// pair p, 3+4g for its crossover point, and 4+4g for mutation (child c, bit
// b at n = c*L + b).
#pragma once
#include <stdint.h>

#include <functional>
#include <vector>

namespace hjga {

double uniform(uint64_t seed, uint64_t stream, uint64_t n);

struct Result {
    uint32_t best_gene = 0;
    double best_time = 0.0;
    int evaluations = 0;                    // distinct genes measured
    std::vector<uint32_t> history;          // [generation][individual] genes
};

// time_of(gene) returns the measured time of a gene in seconds, or a
// non-finite / non-positive value when the measurement failed; such a gene
// counts as kFailTime.
constexpr double kFailTime = 1000.0;

Result run(int gene_bits, int population, int generations, uint64_t seed, double pc, double pm,
           const std::function<double(uint32_t)>& time_of);

}  // namespace hjga

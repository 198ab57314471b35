// Simple GA over offload genes (Sec. 3.3, Sec. 4 and Sec. 5.1.2 of the paper).
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

namespace ofl {

struct GaConfig {
    int M = 12, T = 12;
    double Pc = 0.9, Pm = 0.05, p = 0.5;
    uint64_t seed = 1;
    double deadline_factor = 0.0;
    double timeout_s = 0.0;      // > 0: absolute limit on every run
};

struct GaTrace;
// called after each generation is measured: (generation 1..T, trace so far,
// wall seconds since the search started)
using GaProgress = std::function<void(int, const GaTrace &, double)>;

struct Measurement {
    double t = 0.0;
    int status = 0;   // OFL_ST_*
};

// evaluate(gene, limit_seconds_or_negative) -> measurement of an uncached gene
using Evaluator = std::function<Measurement(const std::vector<uint8_t> &, double)>;
// evaluate_all(genes, limit) -> measurements of a generation's uncached genes
// (first-appearance order), all under the limit taken at the generation start
using BatchEvaluator =
    std::function<std::vector<Measurement>(const std::vector<std::vector<uint8_t>> &, double)>;

struct GaTrace {
    std::vector<std::vector<std::vector<uint8_t>>> pops;   // [gen][m] genes
    std::vector<std::vector<Measurement>> meas;            // [gen][m]
    std::vector<uint8_t> best_gene;
    double best_t = -1.0, best_f = -1.0, t_all0 = -1.0;
    int n_measured = 0;
    double wall_s = 0.0, time_to_best_s = 0.0;
};

// With `batch`, every generation's uncached genes are measured by one call of
// it (the baseline all-zero gene still by `evaluate`).
void run_ga(int a, const GaConfig &cfg, const Evaluator &evaluate, GaTrace &out,
            const BatchEvaluator *batch = nullptr, const GaProgress *progress = nullptr);

double ga_fitness(const Measurement &m, double p);

}  // namespace ofl

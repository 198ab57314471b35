// Simple GA over offload genes (Sec. 3.3, Sec. 4 and Sec. 5.1.2 of the paper).
#pragma once

#include <cstdint>
#include <cstdio>
#include <functional>
#include <string>
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
    uint64_t rng_state = 0;      // state of the GA's random stream after the
                                 // draws of the generations so far
};

// Persistent log of a search (resume after a crash or an interrupted run):
// a first line naming the search (its parameters), then one line per fresh
// measurement in the order taken and one per generation with the random
// stream's state.  Opening an existing log queues its measurements: a
// search with the same parameters takes them from the queue, in order,
// instead of measuring again, which reproduces the interrupted search
// exactly (its trajectory depends only on the seed and the measurements),
// then measures on and appends.  JSON lines; doubles with 17 digits.
class GaLog {
  public:
    ~GaLog();
    // header: the search's identity (a JSON object's members); returns an
    // OFL status (OFL_E_IO when the file cannot be read or written,
    // OFL_E_STATE when it belongs to another search)
    int open(const std::string &path, const std::string &header, std::string &err);
    bool active() const { return f_ != nullptr; }
    // the next queued measurement if it is of gene g: 1 (m filled), 0 (the
    // queue is empty), -1 (the queue holds another gene: not this search)
    int take(const std::vector<uint8_t> &g, Measurement &m);
    void add(const std::vector<uint8_t> &g, const Measurement &m);
    // generation record; during replay it must equal the logged one (false
    // when it does not)
    bool generation(int gen, uint64_t rng_state);
    int replayed() const { return replayed_; }

  private:
    std::FILE *f_ = nullptr;
    std::vector<std::pair<std::vector<uint8_t>, Measurement>> queue_;
    size_t next_ = 0;
    std::vector<uint64_t> gens_;   // logged rng state per generation (index gen - 1)
    int replayed_ = 0;
};

// gate(trace so far) -> whether this generation goes to the batch evaluator
using BatchGate = std::function<bool(const GaTrace &)>;

// With `batch`, every generation's uncached genes are measured by one call of
// it (the baseline all-zero gene still by `evaluate`), except the
// generations for which `gate` (if given) says no: their uncached genes are
// measured one after the other by `evaluate`, each under the limit of that
// moment, as in the search without `batch`.
void run_ga(int a, const GaConfig &cfg, const Evaluator &evaluate, GaTrace &out,
            const BatchEvaluator *batch = nullptr, const GaProgress *progress = nullptr,
            const BatchGate *gate = nullptr);

double ga_fitness(const Measurement &m, double p);

}  // namespace ofl

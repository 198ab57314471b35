// Simple GA over offload genes.
//
// Per the paper (Sec. 3.3, Sec. 4): 0/1 genes, one bit per parallelisable
// loop; M random individuals; each evaluated by running the pattern and
// measuring its time, a faster pattern getting a higher fitness (Sec. 5.1.2:
// time^-1/2); roulette selection by fitness plus the best gene of the
// generation kept as an elite without crossover or mutation; one-point
// crossover with rate Pc; each gene value flipped with rate Pm; stop after T
// generations and answer the best gene; a pattern already measured reuses
// its earlier measurement.
//
// Fixed readings where the paper is silent: T counts the evaluated
// generations including the first; the elite is one of the M (position 0);
// M-1 roulette draws with replacement paired in draw order; crossover point
// uniform in [1, a-1], both children kept, an unpaired last parent copied;
// mutation per bit, elite exempt; failed / timed-out runs get fitness 0; the
// answer is the best fitness over all measurements, earliest on ties.
// Random stream: SplitMix64 (Steele, Lea & Flood 2014) seeded with the GA
// seed, u = (next >> 11) * 2^-53, draws in the order listed above.
#include "ga.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>

#include "../../include/ofl.h"

namespace ofl {

namespace {

class SplitMix64 {
  public:
    explicit SplitMix64(uint64_t seed) : state_(seed) {}
    uint64_t next() {
        uint64_t z = (state_ += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
    uint64_t state() const { return state_; }

  private:
    uint64_t state_;
};

}  // namespace

double ga_fitness(const Measurement &m, double p) {
    if (m.status != OFL_ST_OK || !(m.t > 0.0)) return 0.0;
    return std::pow(m.t, -p);
}

void run_ga(int a, const GaConfig &cfg, const Evaluator &evaluate, GaTrace &out, const BatchEvaluator *batch,
            const GaProgress *progress, const BatchGate *gate) {
    using clk = std::chrono::steady_clock;
    const auto t_start = clk::now();
    out = GaTrace();
    SplitMix64 rng(cfg.seed);
    std::map<std::vector<uint8_t>, Measurement> cache;
    auto elapsed = [&]() { return std::chrono::duration<double>(clk::now() - t_start).count(); };

    auto record = [&](const std::vector<uint8_t> &g, const Measurement &m) {
        out.n_measured++;
        double f = ga_fitness(m, cfg.p);
        if (f > out.best_f) {
            out.best_f = f;
            out.best_t = m.t;
            out.best_gene = g;
            out.time_to_best_s = elapsed();
        }
    };

    if (cfg.deadline_factor > 0.0) {
        std::vector<uint8_t> zero(a, 0);
        Measurement m0 = evaluate(zero, cfg.timeout_s > 0.0 ? cfg.timeout_s : -1.0);
        cache[zero] = m0;
        record(zero, m0);
        if (m0.status == OFL_ST_OK) out.t_all0 = m0.t;
    }

    std::vector<std::vector<uint8_t>> pop(cfg.M, std::vector<uint8_t>(a));
    for (auto &g : pop)
        for (auto &bit : g) bit = (uint8_t)(rng.next() >> 63);

    auto current_limit = [&]() {
        double limit = -1.0;
        if (cfg.deadline_factor > 0.0 && out.best_t > 0.0) {
            limit = cfg.deadline_factor * out.best_t;
            if (out.t_all0 > 0.0 && out.t_all0 < limit) limit = out.t_all0;
        }
        if (cfg.timeout_s > 0.0 && (limit < 0.0 || cfg.timeout_s < limit)) limit = cfg.timeout_s;
        return limit;
    };

    for (int gen = 1; gen <= cfg.T; ++gen) {
        if (batch && (!gate || (*gate)(out))) {
            std::vector<std::vector<uint8_t>> todo;
            for (int m = 0; m < cfg.M; ++m)
                if (!cache.count(pop[m]) && std::find(todo.begin(), todo.end(), pop[m]) == todo.end())
                    todo.push_back(pop[m]);
            if (!todo.empty()) {
                const std::vector<Measurement> got = (*batch)(todo, current_limit());
                for (size_t i = 0; i < todo.size(); ++i) {
                    const Measurement mi = i < got.size() ? got[i] : Measurement{0.0, OFL_ST_FAILED};
                    cache[todo[i]] = mi;
                    record(todo[i], mi);
                }
            }
        }
        std::vector<Measurement> meas(cfg.M);
        std::vector<double> fit(cfg.M);
        for (int m = 0; m < cfg.M; ++m) {
            auto it = cache.find(pop[m]);
            if (it != cache.end()) {
                meas[m] = it->second;
            } else {
                meas[m] = evaluate(pop[m], current_limit());
                cache[pop[m]] = meas[m];
                record(pop[m], meas[m]);
            }
            fit[m] = ga_fitness(meas[m], cfg.p);
        }
        out.pops.push_back(pop);
        out.meas.push_back(meas);
        out.rng_state = rng.state();
        if (progress) (*progress)(gen, out, elapsed());
        if (gen == cfg.T) break;

        int elite = 0;
        for (int m = 1; m < cfg.M; ++m)
            if (fit[m] > fit[elite]) elite = m;
        double total = 0.0;
        for (double f : fit) total += f;

        std::vector<std::vector<uint8_t>> parents;
        parents.reserve(cfg.M - 1);
        for (int d = 0; d < cfg.M - 1; ++d) {
            int pick = cfg.M - 1;
            if (total > 0.0) {
                const double target = rng.uniform() * total;
                double run = 0.0;
                for (int m = 0; m < cfg.M; ++m) {
                    run += fit[m];
                    if (run > target) {
                        pick = m;
                        break;
                    }
                }
            } else {
                pick = (int)(rng.next() % (uint64_t)cfg.M);
            }
            parents.push_back(pop[pick]);
        }
        std::vector<std::vector<uint8_t>> kids;
        size_t k = 0;
        for (; k + 1 < parents.size(); k += 2) {
            std::vector<uint8_t> c1 = parents[k], c2 = parents[k + 1];
            if (rng.uniform() < cfg.Pc && a >= 2) {
                const int cut = 1 + (int)(rng.next() % (uint64_t)(a - 1));
                for (int i = cut; i < a; ++i) {
                    c1[i] = parents[k + 1][i];
                    c2[i] = parents[k][i];
                }
            }
            kids.push_back(std::move(c1));
            kids.push_back(std::move(c2));
        }
        if (k < parents.size()) kids.push_back(parents[k]);
        for (auto &ch : kids)
            for (int i = 0; i < a; ++i)
                if (rng.uniform() < cfg.Pm) ch[i] ^= 1u;
        std::vector<std::vector<uint8_t>> next;
        next.reserve(cfg.M);
        next.push_back(pop[elite]);
        for (auto &ch : kids) next.push_back(std::move(ch));
        pop.swap(next);
    }
    out.wall_s = elapsed();
}

}  // namespace ofl

// Persistent measurement log of a GA search (see GaLog in ga.hpp).
#include <cinttypes>
#include <cstdio>
#include <fstream>
#include <string>

#include "../../include/ofl.h"
#include "ga.hpp"
#include "json.hpp"

namespace ofl {

namespace {

std::string gene_text(const std::vector<uint8_t> &g) {
    std::string s(g.size(), '0');
    for (size_t i = 0; i < g.size(); ++i) s[i] = g[i] ? '1' : '0';
    return s;
}

bool parse_line(const std::string &line, Json &out) {
    std::string err;
    JsonParser jp(line);
    return jp.parse(out, err) && out.kind == Json::Obj;
}

}  // namespace

GaLog::~GaLog() {
    if (f_) std::fclose(f_);
}

int GaLog::open(const std::string &path, const std::string &header, std::string &err) {
    std::ifstream in(path);
    bool have_header = false;
    if (in) {
        std::string line;
        while (std::getline(in, line)) {
            Json j;
            // a line cut short by an interrupted write ends the log
            if (!parse_line(line, j)) break;
            if (!have_header) {
                const Json *id = j.get("search");
                if (!id || id->kind != Json::Str || id->str != header) {
                    err = "GA log " + path + " belongs to another search";
                    return OFL_E_STATE;
                }
                have_header = true;
                continue;
            }
            const Json *g = j.get("gene");
            const Json *gen = j.get("gen");
            if (g && g->kind == Json::Str) {
                const Json *t = j.get("t"), *st = j.get("status");
                if (!t || t->kind != Json::Num || !st || st->kind != Json::Num) break;
                std::vector<uint8_t> gene(g->str.size());
                for (size_t i = 0; i < gene.size(); ++i) gene[i] = g->str[i] == '1' ? 1 : 0;
                queue_.push_back({gene, Measurement{t->num, (int)st->num}});
            } else if (gen && gen->kind == Json::Num) {
                const Json *r = j.get("rng");
                if (!r || r->kind != Json::Str) break;
                gens_.push_back(std::strtoull(r->str.c_str(), nullptr, 16));
            }
        }
    }
    f_ = std::fopen(path.c_str(), have_header ? "a" : "w");
    if (!f_) {
        err = "cannot write GA log " + path;
        return OFL_E_IO;
    }
    if (!have_header) {
        std::fprintf(f_, "{\"search\": \"%s\"}\n", header.c_str());
        std::fflush(f_);
    }
    return OFL_OK;
}

int GaLog::take(const std::vector<uint8_t> &g, Measurement &m) {
    if (next_ >= queue_.size()) return 0;
    if (queue_[next_].first != g) return -1;
    m = queue_[next_++].second;
    ++replayed_;
    return 1;
}

void GaLog::add(const std::vector<uint8_t> &g, const Measurement &m) {
    if (!f_) return;
    std::fprintf(f_, "{\"gene\": \"%s\", \"t\": %.17g, \"status\": %d}\n", gene_text(g).c_str(), m.t, m.status);
    std::fflush(f_);
}

bool GaLog::generation(int gen, uint64_t rng_state) {
    if ((size_t)gen <= gens_.size()) return gens_[gen - 1] == rng_state;
    if (f_) {
        std::fprintf(f_, "{\"gen\": %d, \"rng\": \"%016" PRIx64 "\"}\n", gen, rng_state);
        std::fflush(f_);
    }
    return true;
}

}  // namespace ofl

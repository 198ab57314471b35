// Minimal JSON reader for application descriptions (objects, arrays,
// strings, numbers, true/false/null).  Recursive descent, no dependencies.
#pragma once

#include <cstdlib>
#include <string>
#include <utility>
#include <vector>

namespace ofl {

struct Json {
    enum Kind { Null, Bool, Num, Str, Arr, Obj };
    Kind kind = Null;
    bool b = false;
    double num = 0.0;
    bool is_int = false;
    long long inum = 0;
    std::string str;
    std::vector<Json> arr;
    std::vector<std::pair<std::string, Json>> obj;

    const Json *get(const std::string &key) const {
        if (kind != Obj) return nullptr;
        for (const auto &kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

class JsonParser {
  public:
    explicit JsonParser(const std::string &s) : s_(s) {}

    bool parse(Json &out, std::string &err) {
        pos_ = 0;
        if (!value(out, 0)) {
            err = err_ + " at offset " + std::to_string(pos_);
            return false;
        }
        ws();
        if (pos_ != s_.size()) {
            err = "trailing characters at offset " + std::to_string(pos_);
            return false;
        }
        return true;
    }

  private:
    const std::string &s_;
    size_t pos_ = 0;
    std::string err_;

    void ws() {
        while (pos_ < s_.size() && (s_[pos_] == ' ' || s_[pos_] == '\n' || s_[pos_] == '\t' || s_[pos_] == '\r'))
            ++pos_;
    }
    bool fail(const char *m) {
        err_ = m;
        return false;
    }
    bool lit(const char *w) {
        size_t n = std::char_traits<char>::length(w);
        if (s_.compare(pos_, n, w) != 0) return false;
        pos_ += n;
        return true;
    }
    bool value(Json &v, int depth) {
        if (depth > 64) return fail("nesting too deep");
        ws();
        if (pos_ >= s_.size()) return fail("unexpected end");
        char c = s_[pos_];
        if (c == '{') return object(v, depth);
        if (c == '[') return array(v, depth);
        if (c == '"') {
            v.kind = Json::Str;
            return string(v.str);
        }
        if (lit("true")) { v.kind = Json::Bool; v.b = true; return true; }
        if (lit("false")) { v.kind = Json::Bool; v.b = false; return true; }
        if (lit("null")) { v.kind = Json::Null; return true; }
        return number(v);
    }
    bool object(Json &v, int depth) {
        v.kind = Json::Obj;
        ++pos_;
        ws();
        if (pos_ < s_.size() && s_[pos_] == '}') { ++pos_; return true; }
        for (;;) {
            ws();
            std::string key;
            if (pos_ >= s_.size() || s_[pos_] != '"') return fail("expected key");
            if (!string(key)) return false;
            ws();
            if (pos_ >= s_.size() || s_[pos_] != ':') return fail("expected ':'");
            ++pos_;
            Json child;
            if (!value(child, depth + 1)) return false;
            v.obj.emplace_back(std::move(key), std::move(child));
            ws();
            if (pos_ < s_.size() && s_[pos_] == ',') { ++pos_; continue; }
            if (pos_ < s_.size() && s_[pos_] == '}') { ++pos_; return true; }
            return fail("expected ',' or '}'");
        }
    }
    bool array(Json &v, int depth) {
        v.kind = Json::Arr;
        ++pos_;
        ws();
        if (pos_ < s_.size() && s_[pos_] == ']') { ++pos_; return true; }
        for (;;) {
            Json child;
            if (!value(child, depth + 1)) return false;
            v.arr.push_back(std::move(child));
            ws();
            if (pos_ < s_.size() && s_[pos_] == ',') { ++pos_; continue; }
            if (pos_ < s_.size() && s_[pos_] == ']') { ++pos_; return true; }
            return fail("expected ',' or ']'");
        }
    }
    bool string(std::string &out) {
        ++pos_;  // opening quote
        while (pos_ < s_.size()) {
            char c = s_[pos_++];
            if (c == '"') return true;
            if (c == '\\') {
                if (pos_ >= s_.size()) return fail("bad escape");
                char e = s_[pos_++];
                switch (e) {
                case '"': out += '"'; break;
                case '\\': out += '\\'; break;
                case '/': out += '/'; break;
                case 'n': out += '\n'; break;
                case 't': out += '\t'; break;
                case 'r': out += '\r'; break;
                case 'b': out += '\b'; break;
                case 'f': out += '\f'; break;
                case 'u': {
                    if (pos_ + 4 > s_.size()) return fail("bad \\u escape");
                    unsigned code = (unsigned)std::strtoul(s_.substr(pos_, 4).c_str(), nullptr, 16);
                    pos_ += 4;
                    if (code < 0x80) out += (char)code;
                    else if (code < 0x800) {
                        out += (char)(0xC0 | (code >> 6));
                        out += (char)(0x80 | (code & 0x3F));
                    } else {
                        out += (char)(0xE0 | (code >> 12));
                        out += (char)(0x80 | ((code >> 6) & 0x3F));
                        out += (char)(0x80 | (code & 0x3F));
                    }
                    break;
                }
                default: return fail("bad escape");
                }
            } else {
                out += c;
            }
        }
        return fail("unterminated string");
    }
    bool number(Json &v) {
        size_t start = pos_;
        if (pos_ < s_.size() && (s_[pos_] == '-' || s_[pos_] == '+')) ++pos_;
        bool frac = false;
        while (pos_ < s_.size()) {
            char c = s_[pos_];
            if (c >= '0' && c <= '9') { ++pos_; continue; }
            if (c == '.' || c == 'e' || c == 'E' || ((c == '-' || c == '+') && frac)) {
                frac = true;
                ++pos_;
                continue;
            }
            break;
        }
        if (pos_ == start) return fail("unexpected character");
        std::string t = s_.substr(start, pos_ - start);
        char *end = nullptr;
        v.kind = Json::Num;
        v.num = std::strtod(t.c_str(), &end);
        if (!end || *end) return fail("bad number");
        if (!frac) {
            v.is_int = true;
            v.inum = std::strtoll(t.c_str(), nullptr, 10);
        }
        return true;
    }
};

}  // namespace ofl

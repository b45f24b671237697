// Autotune results on disk: a small JSON document holding the library
// version, the device's architecture name and compute-unit count, and one
// record per tuned plan shape (its key and the forward schedule chosen).
// The reader accepts the subset of JSON the writer produces (objects,
// arrays, strings, integers, booleans, null), rejects anything malformed
// and never reads past its input.
#include <cctype>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <utility>
#include <vector>

#include "sg_internal.hpp"

namespace sg {

namespace {

void put_string(std::string& out, const std::string& s)
{
    out += '"';
    for (const char ch : s) {
        const unsigned char c = (unsigned char)ch;
        if (c == '"' || c == '\\') {
            out += '\\';
            out += ch;
        } else if (c >= 0x20 && c < 0x7f) {
            out += ch;
        }   // control and non-ASCII bytes are dropped (names are ASCII)
    }
    out += '"';
}

struct JValue {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    bool b = false;
    int64_t num = 0;
    std::string str;
    std::vector<JValue> arr;
    std::vector<std::pair<std::string, JValue>> obj;

    const JValue* get(const char* name) const
    {
        if (kind != OBJ) return nullptr;
        for (const auto& kv : obj)
            if (kv.first == name) return &kv.second;
        return nullptr;
    }
};

class Parser {
public:
    explicit Parser(const std::string& text) : s_(text) {}

    bool document(JValue& v)
    {
        if (!value(v, 0)) return false;
        skip();
        return i_ == s_.size();
    }

private:
    static constexpr int kMaxDepth = 8;
    const std::string& s_;
    size_t i_ = 0;

    void skip()
    {
        while (i_ < s_.size() && (s_[i_] == ' ' || s_[i_] == '\n' || s_[i_] == '\r' || s_[i_] == '\t')) ++i_;
    }
    bool literal(const char* word)
    {
        size_t k = 0;
        while (word[k]) {
            if (i_ + k >= s_.size() || s_[i_ + k] != word[k]) return false;
            ++k;
        }
        i_ += k;
        return true;
    }
    bool string(std::string& out)
    {
        if (i_ >= s_.size() || s_[i_] != '"') return false;
        ++i_;
        while (i_ < s_.size()) {
            const char c = s_[i_++];
            if (c == '"') return true;
            if ((unsigned char)c < 0x20) return false;
            if (c == '\\') {
                if (i_ >= s_.size()) return false;
                const char e = s_[i_++];
                if (e == '"' || e == '\\' || e == '/') out += e;
                else if (e == 'n') out += '\n';
                else if (e == 't') out += '\t';
                else return false;   // other escapes never written
            } else {
                out += c;
            }
        }
        return false;
    }
    bool number(int64_t& out)
    {
        bool neg = false;
        if (i_ < s_.size() && s_[i_] == '-') {
            neg = true;
            ++i_;
        }
        if (i_ >= s_.size() || !std::isdigit((unsigned char)s_[i_])) return false;
        uint64_t v = 0;
        int digits = 0;
        while (i_ < s_.size() && std::isdigit((unsigned char)s_[i_])) {
            if (++digits > 18) return false;   // keeps v below 10^18
            v = v * 10 + (uint64_t)(s_[i_++] - '0');
        }
        if (i_ < s_.size() && (s_[i_] == '.' || s_[i_] == 'e' || s_[i_] == 'E')) return false;   // integers only
        out = neg ? -(int64_t)v : (int64_t)v;
        return true;
    }
    bool value(JValue& v, int depth)
    {
        if (depth > kMaxDepth) return false;
        skip();
        if (i_ >= s_.size()) return false;
        const char c = s_[i_];
        if (c == '{') {
            v.kind = JValue::OBJ;
            ++i_;
            skip();
            if (i_ < s_.size() && s_[i_] == '}') {
                ++i_;
                return true;
            }
            for (;;) {
                skip();
                std::string name;
                if (!string(name)) return false;
                skip();
                if (i_ >= s_.size() || s_[i_] != ':') return false;
                ++i_;
                JValue member;
                if (!value(member, depth + 1)) return false;
                v.obj.emplace_back(std::move(name), std::move(member));
                skip();
                if (i_ >= s_.size()) return false;
                if (s_[i_] == ',') {
                    ++i_;
                    continue;
                }
                if (s_[i_] == '}') {
                    ++i_;
                    return true;
                }
                return false;
            }
        }
        if (c == '[') {
            v.kind = JValue::ARR;
            ++i_;
            skip();
            if (i_ < s_.size() && s_[i_] == ']') {
                ++i_;
                return true;
            }
            for (;;) {
                JValue item;
                if (!value(item, depth + 1)) return false;
                v.arr.push_back(std::move(item));
                skip();
                if (i_ >= s_.size()) return false;
                if (s_[i_] == ',') {
                    ++i_;
                    continue;
                }
                if (s_[i_] == ']') {
                    ++i_;
                    return true;
                }
                return false;
            }
        }
        if (c == '"') {
            v.kind = JValue::STR;
            return string(v.str);
        }
        if (literal("true")) {
            v.kind = JValue::BOOL;
            v.b = true;
            return true;
        }
        if (literal("false")) {
            v.kind = JValue::BOOL;
            return true;
        }
        if (literal("null")) return true;
        v.kind = JValue::NUM;
        return number(v.num);
    }
};

bool get_int(const JValue& o, const char* name, int64_t lo, int64_t hi, int& out)
{
    const JValue* v = o.get(name);
    if (!v || v->kind != JValue::NUM || v->num < lo || v->num > hi) return false;
    out = (int)v->num;
    return true;
}

bool get_str(const JValue& o, const char* name, std::string& out)
{
    const JValue* v = o.get(name);
    if (!v || v->kind != JValue::STR) return false;
    out = v->str;
    return true;
}

}  // namespace

std::string tune_file_write(const TuneFile& f)
{
    std::string out = "{\n  \"format\": ";
    put_string(out, kTuneFormat);
    out += ",\n  \"version\": ";
    put_string(out, f.version);
    out += ",\n  \"arch\": ";
    put_string(out, f.arch);
    out += ",\n  \"compute_units\": " + std::to_string(f.compute_units) + ",\n  \"entries\": [";
    for (size_t k = 0; k < f.entries.size(); ++k) {
        const TuneRecord& r = f.entries[k];
        out += k ? ",\n    {\"key\": " : "\n    {\"key\": ";
        put_string(out, r.key);
        out += ", \"coords_per_lane\": " + std::to_string(r.cpl) + ", \"max_group\": " + std::to_string(r.gmax) +
               ", \"cost_scaled\": " + std::to_string(r.cost_scaled) + ", \"persistent\": " +
               std::to_string(r.persistent) + ", \"balanced\": " + std::to_string(r.balanced) +
               ", \"graph\": " + std::to_string(r.graph) + "}";
    }
    out += f.entries.empty() ? "]\n}\n" : "\n  ]\n}\n";
    return out;
}

bool tune_file_read(const std::string& text, TuneFile& f, std::string& err)
{
    JValue doc;
    Parser ps(text);
    if (!ps.document(doc) || doc.kind != JValue::OBJ) {
        err = "not a JSON object";
        return false;
    }
    std::string format;
    if (!get_str(doc, "format", format) || format != kTuneFormat) {
        err = "not an autotune file of this format";
        return false;
    }
    if (!get_str(doc, "version", f.version) || !get_str(doc, "arch", f.arch) ||
        !get_int(doc, "compute_units", 1, 1 << 20, f.compute_units)) {
        err = "missing version, arch or compute_units";
        return false;
    }
    const JValue* entries = doc.get("entries");
    if (!entries || entries->kind != JValue::ARR) {
        err = "missing entries";
        return false;
    }
    f.entries.clear();
    for (const JValue& e : entries->arr) {
        TuneRecord r;
        if (e.kind != JValue::OBJ || !get_str(e, "key", r.key) || r.key.empty() || r.key.size() > 128 ||
            !get_int(e, "coords_per_lane", 1, 64, r.cpl) || !get_int(e, "max_group", 1, 4, r.gmax) || r.gmax == 3 ||
            !get_int(e, "cost_scaled", 0, 1, r.cost_scaled) || !get_int(e, "persistent", 0, 1, r.persistent) ||
            !get_int(e, "balanced", 0, 8, r.balanced) || !get_int(e, "graph", 0, 1, r.graph)) {
            err = "malformed entry " + std::to_string(f.entries.size());
            return false;
        }
        f.entries.push_back(std::move(r));
    }
    return true;
}

}  // namespace sg

// Autotune cache file: a small recursive-descent reader for the JSON subset the
// cache uses (objects, arrays, strings, numbers, true / false / null) and its
// writer.  Host code only.
#include "hh_tune_cache.h"

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

namespace hh {

namespace {

struct Reader {
    const std::string& s;
    size_t i = 0;
    std::string err;

    explicit Reader(const std::string& text) : s(text) {}

    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool fail(const char* what) {
        if (err.empty()) {
            char buf[160];
            std::snprintf(buf, sizeof(buf), "%s at byte %zu", what, i);
            err = buf;
        }
        return false;
    }
    bool eat(char ch) {
        ws();
        if (i < s.size() && s[i] == ch) {
            ++i;
            return true;
        }
        return false;
    }
    bool string(std::string& out) {
        ws();
        if (i >= s.size() || s[i] != '"') return fail("expected a string");
        ++i;
        out.clear();
        while (i < s.size() && s[i] != '"') {
            char ch = s[i++];
            if (ch == '\\') {
                if (i >= s.size()) return fail("unterminated escape");
                const char e = s[i++];
                switch (e) {
                    case '"': case '\\': case '/': ch = e; break;
                    case 'n': ch = '\n'; break;
                    case 't': ch = '\t'; break;
                    case 'r': ch = '\r'; break;
                    case 'b': ch = '\b'; break;
                    case 'f': ch = '\f'; break;
                    default: return fail("unsupported escape in a string");
                }
            }
            out.push_back(ch);
        }
        if (i >= s.size()) return fail("unterminated string");
        ++i;
        return true;
    }
    bool number(double& out) {
        ws();
        const char* p = s.c_str() + i;
        char* end = nullptr;
        out = std::strtod(p, &end);
        if (end == p) return fail("expected a number");
        i += (size_t)(end - p);
        return true;
    }
    bool integer(int& out) {
        double d;
        if (!number(d)) return false;
        if (!(d >= -1e9 && d <= 1e9) || d != std::floor(d)) return fail("expected an integer");
        out = (int)d;
        return true;
    }
    bool int_array(std::vector<int>& out) {
        out.clear();
        if (!eat('[')) return fail("expected an array");
        if (eat(']')) return true;
        do {
            int v;
            if (!integer(v)) return false;
            out.push_back(v);
        } while (eat(','));
        return eat(']') || fail("expected ']'");
    }
    // any value, discarded (fields this version does not know)
    bool skip(int depth = 0) {
        if (depth > 32) return fail("nesting too deep");
        ws();
        if (i >= s.size()) return fail("unexpected end");
        if (s[i] == '"') {
            std::string tmp;
            return string(tmp);
        }
        if (s[i] == '{' || s[i] == '[') {
            const char close = s[i] == '{' ? '}' : ']';
            const bool obj = s[i] == '{';
            ++i;
            if (eat(close)) return true;
            do {
                if (obj) {
                    std::string k;
                    if (!string(k) || !eat(':')) return fail("expected a member");
                }
                if (!skip(depth + 1)) return false;
            } while (eat(','));
            return eat(close) || fail("expected the end of a container");
        }
        for (const char* lit : {"true", "false", "null"})
            if (s.compare(i, std::strlen(lit), lit) == 0) {
                i += std::strlen(lit);
                return true;
            }
        double d;
        return number(d);
    }
    bool entry(TuneEntry& e) {
        if (!eat('{')) return fail("expected an entry object");
        if (eat('}')) return true;
        do {
            std::string k;
            if (!string(k) || !eat(':')) return fail("expected a member of an entry");
            bool ok;
            if (k == "block") ok = integer(e.block);
            else if (k == "zb") ok = integer(e.zb);
            else if (k == "zb_down") ok = int_array(e.zb_down);
            else if (k == "zb_up") ok = int_array(e.zb_up);
            else if (k == "dn_region") ok = int_array(e.dn_region);
            else if (k == "step_ms") ok = number(e.step_ms);
            else if (k == "default_step_ms") ok = number(e.default_step_ms);
            else ok = skip();
            if (!ok) return false;
        } while (eat(','));
        return eat('}') || fail("expected '}' after an entry");
    }
};

void put_array(std::ostringstream& o, const std::vector<int>& v) {
    o << '[';
    for (size_t j = 0; j < v.size(); ++j) o << (j ? ", " : "") << v[j];
    o << ']';
}

void put_string(std::ostringstream& o, const std::string& v) {
    o << '"';
    for (char ch : v) {
        if (ch == '"' || ch == '\\') o << '\\';
        o << ch;
    }
    o << '"';
}

}  // namespace

bool tune_cache_read(const char* path, std::map<std::string, TuneEntry>& out, std::string& err) {
    out.clear();
    std::ifstream f(path, std::ios::binary);
    if (!f) return true;  // no file yet: an empty cache
    std::stringstream buf;
    buf << f.rdbuf();
    const std::string text = buf.str();
    Reader r(text);
    r.ws();
    if (r.i == text.size()) return true;  // empty file
    bool ok = r.eat('{');
    if (!ok) r.fail("the cache file is not a JSON object");
    if (ok && !r.eat('}')) {
        do {
            std::string key;
            TuneEntry e;
            if (!r.string(key) || !r.eat(':') || !r.entry(e)) {
                ok = false;
                break;
            }
            out[key] = e;
        } while (r.eat(','));
        if (ok && !r.eat('}')) ok = r.fail("expected '}' at the end of the cache object");
    }
    if (ok) {
        r.ws();
        if (r.i != text.size()) ok = r.fail("trailing data after the cache object");
    }
    if (!ok) {
        err = std::string(path) + ": " + r.err;
        out.clear();
    }
    return ok;
}

bool tune_cache_write(const char* path, const std::map<std::string, TuneEntry>& m, std::string& err) {
    std::ostringstream o;
    o << "{\n";
    size_t n = 0;
    for (const auto& kv : m) {
        const TuneEntry& e = kv.second;
        o << "  ";
        put_string(o, kv.first);
        o << ": {\"block\": " << e.block << ", \"zb\": " << e.zb << ", \"zb_down\": ";
        put_array(o, e.zb_down);
        o << ", \"zb_up\": ";
        put_array(o, e.zb_up);
        o << ", \"dn_region\": ";
        put_array(o, e.dn_region);
        char num[96];
        std::snprintf(num, sizeof(num), ", \"step_ms\": %.6g, \"default_step_ms\": %.6g}", e.step_ms,
                      e.default_step_ms);
        o << num << (++n < m.size() ? ",\n" : "\n");
    }
    o << "}\n";
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
        if (!f) {
            err = "cannot write " + tmp;
            return false;
        }
        const std::string text = o.str();
        f.write(text.data(), (std::streamsize)text.size());
        if (!f) {
            err = "cannot write " + tmp;
            return false;
        }
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        err = "cannot rename " + tmp + " to " + path;
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace hh

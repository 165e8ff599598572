// gdi_tunecache.cpp -- JSON reading and writing of the autotuner's cache (format in
// gdi_tunecache.h). A small recursive-descent reader: objects, arrays, strings with
// the standard escapes, numbers, true/false/null; nesting is bounded.
#include "gdi_tunecache.h"

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <unistd.h>

#include <cmath>
#include <fstream>
#include <sstream>

namespace gdi_tunecache {
namespace {

const int kMaxDepth = 32;

struct Reader {
    const std::string &s;
    size_t i = 0;
    std::string err;

    explicit Reader(const std::string &t) : s(t) {}

    bool fail(const std::string &m)
    {
        if (err.empty()) err = m + " at byte " + std::to_string(i);
        return false;
    }
    void ws()
    {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\t' || s[i] == '\n' || s[i] == '\r')) ++i;
    }
    bool eat(char c)
    {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool hex4(uint32_t *u)
    {
        if (i + 4 > s.size()) return fail("truncated \\u escape");
        uint32_t v = 0;
        for (int k = 0; k < 4; ++k) {
            const char c = s[i++];
            v <<= 4;
            if (c >= '0' && c <= '9') v |= (uint32_t)(c - '0');
            else if (c >= 'a' && c <= 'f') v |= (uint32_t)(c - 'a' + 10);
            else if (c >= 'A' && c <= 'F') v |= (uint32_t)(c - 'A' + 10);
            else return fail("bad \\u escape");
        }
        *u = v;
        return true;
    }
    static void utf8(uint32_t cp, std::string *o)
    {
        if (cp < 0x80) {
            o->push_back((char)cp);
        } else if (cp < 0x800) {
            o->push_back((char)(0xC0 | (cp >> 6)));
            o->push_back((char)(0x80 | (cp & 0x3F)));
        } else if (cp < 0x10000) {
            o->push_back((char)(0xE0 | (cp >> 12)));
            o->push_back((char)(0x80 | ((cp >> 6) & 0x3F)));
            o->push_back((char)(0x80 | (cp & 0x3F)));
        } else {
            o->push_back((char)(0xF0 | (cp >> 18)));
            o->push_back((char)(0x80 | ((cp >> 12) & 0x3F)));
            o->push_back((char)(0x80 | ((cp >> 6) & 0x3F)));
            o->push_back((char)(0x80 | (cp & 0x3F)));
        }
    }
    bool str(std::string *o)
    {
        ws();
        if (i >= s.size() || s[i] != '"') return fail("expected a string");
        ++i;
        o->clear();
        while (i < s.size()) {
            const char c = s[i++];
            if (c == '"') return true;
            if ((unsigned char)c < 0x20) return fail("control character in a string");
            if (c != '\\') {
                o->push_back(c);
                continue;
            }
            if (i >= s.size()) break;
            const char e = s[i++];
            switch (e) {
            case '"': o->push_back('"'); break;
            case '\\': o->push_back('\\'); break;
            case '/': o->push_back('/'); break;
            case 'b': o->push_back('\b'); break;
            case 'f': o->push_back('\f'); break;
            case 'n': o->push_back('\n'); break;
            case 'r': o->push_back('\r'); break;
            case 't': o->push_back('\t'); break;
            case 'u': {
                uint32_t u = 0;
                if (!hex4(&u)) return false;
                if (u >= 0xD800 && u < 0xDC00) {  // a surrogate pair
                    uint32_t lo = 0;
                    if (i + 2 > s.size() || s[i] != '\\' || s[i + 1] != 'u') return fail("lone surrogate");
                    i += 2;
                    if (!hex4(&lo)) return false;
                    if (lo < 0xDC00 || lo >= 0xE000) return fail("bad surrogate pair");
                    u = 0x10000 + ((u - 0xD800) << 10) + (lo - 0xDC00);
                } else if (u >= 0xDC00 && u < 0xE000) {
                    return fail("lone surrogate");
                }
                utf8(u, o);
                break;
            }
            default: return fail("bad escape");
            }
        }
        return fail("unterminated string");
    }
    bool num(double *v)
    {
        ws();
        const size_t b = i;
        if (i < s.size() && s[i] == '-') ++i;
        if (i >= s.size() || s[i] < '0' || s[i] > '9') return fail("expected a number");
        while (i < s.size() && ((s[i] >= '0' && s[i] <= '9') || s[i] == '.' || s[i] == 'e' || s[i] == 'E' ||
                                s[i] == '+' || s[i] == '-'))
            ++i;
        const std::string t = s.substr(b, i - b);
        char *end = nullptr;
        *v = strtod(t.c_str(), &end);
        if (!end || *end != '\0' || !std::isfinite(*v)) return fail("bad number");
        return true;
    }
    bool word(const char *w)
    {
        size_t k = 0;
        while (w[k]) {
            if (i + k >= s.size() || s[i + k] != w[k]) return fail("bad literal");
            ++k;
        }
        i += k;
        return true;
    }
    // skips one value of any kind
    bool skip(int depth)
    {
        if (depth > kMaxDepth) return fail("nesting too deep");
        ws();
        if (i >= s.size()) return fail("unexpected end");
        const char c = s[i];
        if (c == '"') {
            std::string t;
            return str(&t);
        }
        if (c == '{') {
            ++i;
            if (eat('}')) return true;
            do {
                std::string k;
                if (!str(&k) || !eat(':') || !skip(depth + 1)) return fail("bad object");
            } while (eat(','));
            return eat('}') || fail("expected '}'");
        }
        if (c == '[') {
            ++i;
            if (eat(']')) return true;
            do {
                if (!skip(depth + 1)) return false;
            } while (eat(','));
            return eat(']') || fail("expected ']'");
        }
        if (c == 't') return word("true");
        if (c == 'f') return word("false");
        if (c == 'n') return word("null");
        double v = 0;
        return num(&v);
    }
    bool fields(Fields *f)
    {
        if (!eat('{')) return fail("an entry must be an object");
        if (eat('}')) return true;
        do {
            std::string k;
            double v = 0;
            if (!str(&k) || !eat(':') || !num(&v)) return fail("entry fields must be numbers");
            (*f)[k] = v;
        } while (eat(','));
        return eat('}') || fail("expected '}'");
    }
    bool entries(Table *t)
    {
        if (!eat('{')) return fail("\"entries\" must be an object");
        if (eat('}')) return true;
        do {
            std::string k;
            Fields f;
            if (!str(&k) || !eat(':') || !fields(&f)) return false;
            (*t)[k] = f;
        } while (eat(','));
        return eat('}') || fail("expected '}'");
    }
};

void put_string(const std::string &k, std::string *o)
{
    o->push_back('"');
    for (const char c : k) {
        const unsigned char u = (unsigned char)c;
        if (c == '"' || c == '\\') {
            o->push_back('\\');
            o->push_back(c);
        } else if (u < 0x20) {
            char b[8];
            snprintf(b, sizeof b, "\\u%04x", u);
            *o += b;
        } else {
            o->push_back(c);
        }
    }
    o->push_back('"');
}

void put_number(double v, std::string *o)
{
    char b[40];
    if (std::isfinite(v) && v == std::floor(v) && std::fabs(v) < 9.0e15)
        snprintf(b, sizeof b, "%lld", (long long)v);
    else if (std::isfinite(v))
        snprintf(b, sizeof b, "%.17g", v);
    else
        snprintf(b, sizeof b, "0");  // JSON has no infinities; the reader rejects none of ours
    *o += b;
}

}  // namespace

int parse(const std::string &text, Table *out, std::string *err)
{
    Reader r(text);
    Table got;
    bool have_format = false, ok = r.eat('{');
    if (!ok) r.fail("expected a JSON object");
    if (ok && !r.eat('}')) {
        do {
            std::string k;
            if (!(ok = r.str(&k) && r.eat(':'))) break;
            if (k == "format") {
                std::string f;
                if (!(ok = r.str(&f))) break;
                if (f != "gdi-tune-1") {
                    ok = r.fail("unknown format \"" + f + "\"");
                    break;
                }
                have_format = true;
            } else if (k == "entries") {
                if (!(ok = r.entries(&got))) break;
            } else if (!(ok = r.skip(1))) {
                break;
            }
        } while (r.eat(','));
        if (ok) ok = r.eat('}') || r.fail("expected '}'");
    }
    if (ok) {
        r.ws();
        if (r.i != text.size()) ok = r.fail("trailing characters");
    }
    if (ok && !have_format) ok = r.fail("no \"format\" member");
    if (!ok) {
        if (err) *err = r.err.empty() ? std::string("malformed tuning cache") : r.err;
        return -1;
    }
    for (auto &e : got) (*out)[e.first] = e.second;
    return 0;
}

std::string dump(const Table &t)
{
    std::string o = "{\"format\": \"gdi-tune-1\",\n \"entries\": {";
    bool first = true;
    for (const auto &e : t) {
        o += first ? "\n  " : ",\n  ";
        first = false;
        put_string(e.first, &o);
        o += ": {";
        bool f1 = true;
        for (const auto &f : e.second) {
            if (!f1) o += ", ";
            f1 = false;
            put_string(f.first, &o);
            o += ": ";
            put_number(f.second, &o);
        }
        o += "}";
    }
    o += "\n }\n}\n";
    return o;
}

bool read_file(const std::string &path, std::string *text)
{
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    std::ostringstream ss;
    ss << f.rdbuf();
    if (f.bad()) return false;
    *text = ss.str();
    return true;
}

bool write_file(const std::string &path, const std::string &text)
{
    const std::string tmp = path + ".tmp." + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return false;
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    if (fclose(f) != 0 || !ok) {
        remove(tmp.c_str());
        return false;
    }
    if (rename(tmp.c_str(), path.c_str()) != 0) {
        remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace gdi_tunecache

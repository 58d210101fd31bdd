// Minimal JSON reader for model descriptions (objects, arrays, numbers,
// strings, true/false/null). Throws JsonError with a position on bad input:
// malformed text, nesting deeper than MAX_DEPTH, and numbers that are not
// finite or not in JSON's decimal form.
#pragma once

#include <cmath>
#include <cstdlib>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace nufold {

struct JsonError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

struct Json {
  enum Kind { Null, Bool, Number, String, Array, Object } kind = Null;
  bool b = false;
  double num = 0.0;
  std::string str;
  std::vector<Json> arr;
  std::map<std::string, Json> obj;

  bool is_null() const { return kind == Null; }
  bool has(const std::string& k) const { return kind == Object && obj.count(k); }
  const Json& at(const std::string& k) const {
    if (kind != Object) throw JsonError("expected an object while looking up '" + k + "'");
    auto it = obj.find(k);
    if (it == obj.end()) throw JsonError("missing key '" + k + "'");
    return it->second;
  }
  // returns a null value for a missing key
  const Json& get(const std::string& k) const {
    static const Json null_value;
    if (kind != Object) return null_value;
    auto it = obj.find(k);
    return it == obj.end() ? null_value : it->second;
  }
  const std::vector<Json>& array() const {
    if (kind != Array) throw JsonError("expected an array");
    return arr;
  }
  double number() const {
    if (kind != Number) throw JsonError("expected a number");
    return num;
  }
  const std::string& string() const {
    if (kind != String) throw JsonError("expected a string");
    return str;
  }
  bool boolean() const {
    if (kind != Bool) throw JsonError("expected true/false");
    return b;
  }
};

class JsonParser {
 public:
  static constexpr int MAX_DEPTH = 256;
  explicit JsonParser(const char* s) : p_(s), start_(s) {}

  Json parse() {
    Json v = value();
    ws();
    if (*p_) fail("trailing characters");
    return v;
  }

 private:
  const char* p_;
  const char* start_;
  int depth_ = 0;

  [[noreturn]] void fail(const std::string& what) {
    throw JsonError("JSON: " + what + " at offset " + std::to_string(p_ - start_));
  }
  void ws() {
    while (*p_ == ' ' || *p_ == '\n' || *p_ == '\t' || *p_ == '\r') ++p_;
  }
  bool lit(const char* w) {
    size_t n = 0;
    while (w[n]) ++n;
    for (size_t i = 0; i < n; ++i)
      if (p_[i] != w[i]) return false;
    p_ += n;
    return true;
  }
  Json value() {
    ws();
    Json v;
    char c = *p_;
    if ((c == '{' || c == '[') && ++depth_ > MAX_DEPTH) fail("nesting deeper than " + std::to_string(MAX_DEPTH));
    if (c == '{') {
      v.kind = Json::Object;
      ++p_;
      ws();
      if (*p_ == '}') { ++p_; --depth_; return v; }
      for (;;) {
        ws();
        if (*p_ != '"') fail("expected a key string");
        std::string k = strlit();
        ws();
        if (*p_ != ':') fail("expected ':'");
        ++p_;
        v.obj[k] = value();
        ws();
        if (*p_ == ',') { ++p_; continue; }
        if (*p_ == '}') { ++p_; break; }
        fail("expected ',' or '}'");
      }
      --depth_;
    } else if (c == '[') {
      v.kind = Json::Array;
      ++p_;
      ws();
      if (*p_ == ']') { ++p_; --depth_; return v; }
      for (;;) {
        v.arr.push_back(value());
        ws();
        if (*p_ == ',') { ++p_; continue; }
        if (*p_ == ']') { ++p_; break; }
        fail("expected ',' or ']'");
      }
      --depth_;
    } else if (c == '"') {
      v.kind = Json::String;
      v.str = strlit();
    } else if (lit("true")) {
      v.kind = Json::Bool; v.b = true;
    } else if (lit("false")) {
      v.kind = Json::Bool; v.b = false;
    } else if (lit("null")) {
      v.kind = Json::Null;
    } else if (lit("NaN") || lit("Infinity") || lit("-Infinity")) {
      fail("non-finite numbers are not allowed");
    } else if (c == '-' || (c >= '0' && c <= '9')) {
      // JSON's decimal form only (strtod alone would also take inf, nan and
      // hexadecimal forms), and a finite value
      const char* q = p_;
      while ((*q >= '0' && *q <= '9') || *q == '-' || *q == '+' || *q == '.' || *q == 'e' || *q == 'E') ++q;
      const std::string tok(p_, q);
      char* end = nullptr;
      v.kind = Json::Number;
      v.num = std::strtod(tok.c_str(), &end);
      if (end != tok.c_str() + tok.size() || tok.empty()) fail("bad number");
      if (!std::isfinite(v.num)) fail("number out of range");
      p_ = q;
    } else {
      fail("unexpected character");
    }
    return v;
  }
  std::string strlit() {
    ++p_;  // opening quote
    std::string s;
    while (*p_ && *p_ != '"') {
      if (*p_ == '\\') {
        ++p_;
        switch (*p_) {
          case '"': s += '"'; break;
          case '\\': s += '\\'; break;
          case '/': s += '/'; break;
          case 'n': s += '\n'; break;
          case 't': s += '\t'; break;
          case 'r': s += '\r'; break;
          case 'b': s += '\b'; break;
          case 'f': s += '\f'; break;
          case 'u': {
            unsigned cp = 0;
            for (int i = 1; i <= 4; ++i) {
              char h = p_[i];
              cp <<= 4;
              if (h >= '0' && h <= '9') cp |= h - '0';
              else if (h >= 'a' && h <= 'f') cp |= h - 'a' + 10;
              else if (h >= 'A' && h <= 'F') cp |= h - 'A' + 10;
              else fail("bad \\u escape");
            }
            p_ += 4;
            if (cp < 0x80) s += char(cp);
            else if (cp < 0x800) { s += char(0xC0 | (cp >> 6)); s += char(0x80 | (cp & 0x3F)); }
            else { s += char(0xE0 | (cp >> 12)); s += char(0x80 | ((cp >> 6) & 0x3F)); s += char(0x80 | (cp & 0x3F)); }
            break;
          }
          default: fail("bad escape");
        }
        ++p_;
      } else {
        s += *p_++;
      }
    }
    if (*p_ != '"') fail("unterminated string");
    ++p_;
    return s;
  }
};

inline Json parse_json(const char* s) { return JsonParser(s).parse(); }

}  // namespace nufold

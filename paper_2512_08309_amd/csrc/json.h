// Minimal JSON reader for the weight-file header (objects, arrays, strings,
// numbers, true/false/null).  Throws td::Error{TD_E_FORMAT} on bad input.
#pragma once

#include <cstdlib>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "td_error.h"

namespace td {

struct Json {
  enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
  bool b = false;
  double n = 0;
  std::string s;
  std::vector<Json> a;
  std::map<std::string, Json> o;

  const Json& at(const std::string& k) const {
    auto it = o.find(k);
    if (kind != Obj || it == o.end()) throw Error{-5, "weight header: missing key '" + k + "'"};
    return it->second;
  }
  bool has(const std::string& k) const { return kind == Obj && o.count(k); }
  double num() const {
    if (kind != Num) throw Error{-5, "weight header: expected a number"};
    return n;
  }
  long long integer() const {
    double v = num();
    // range first: converting a double outside int64 is undefined
    if (!(v >= -9.0e18 && v <= 9.0e18) || v != (double)(long long)v)
      throw Error{-5, "weight header: expected an integer"};
    return (long long)v;
  }
  const std::string& str() const {
    if (kind != Str) throw Error{-5, "weight header: expected a string"};
    return s;
  }
  bool boolean() const {
    if (kind != Bool) throw Error{-5, "weight header: expected a boolean"};
    return b;
  }
  const std::vector<Json>& arr() const {
    if (kind != Arr) throw Error{-5, "weight header: expected an array"};
    return a;
  }
};

class JsonParser {
 public:
  explicit JsonParser(const std::string& t) : t_(t) {}
  Json parse() {
    Json v = value();
    ws();
    if (i_ != t_.size()) fail("trailing characters");
    return v;
  }

 private:
  const std::string& t_;
  size_t i_ = 0;
  int depth_ = 0;

  [[noreturn]] void fail(const char* what) {
    throw Error{-5, std::string("weight header JSON: ") + what + " at byte " + std::to_string(i_)};
  }
  void ws() {
    while (i_ < t_.size() && (t_[i_] == ' ' || t_[i_] == '\n' || t_[i_] == '\r' || t_[i_] == '\t')) ++i_;
  }
  bool lit(const char* w) {
    size_t n = std::char_traits<char>::length(w);
    if (t_.compare(i_, n, w) == 0) {
      i_ += n;
      return true;
    }
    return false;
  }
  Json value() {
    if (++depth_ > 64) fail("nesting too deep");
    ws();
    if (i_ >= t_.size()) fail("unexpected end");
    Json v;
    char c = t_[i_];
    if (c == '{') {
      v.kind = Json::Obj;
      ++i_;
      ws();
      if (i_ < t_.size() && t_[i_] == '}') {
        ++i_;
      } else {
        for (;;) {
          ws();
          if (i_ >= t_.size() || t_[i_] != '"') fail("expected key");
          std::string k = string();
          ws();
          if (i_ >= t_.size() || t_[i_] != ':') fail("expected ':'");
          ++i_;
          v.o[k] = value();
          ws();
          if (i_ < t_.size() && t_[i_] == ',') { ++i_; continue; }
          if (i_ < t_.size() && t_[i_] == '}') { ++i_; break; }
          fail("expected ',' or '}'");
        }
      }
    } else if (c == '[') {
      v.kind = Json::Arr;
      ++i_;
      ws();
      if (i_ < t_.size() && t_[i_] == ']') {
        ++i_;
      } else {
        for (;;) {
          v.a.push_back(value());
          ws();
          if (i_ < t_.size() && t_[i_] == ',') { ++i_; continue; }
          if (i_ < t_.size() && t_[i_] == ']') { ++i_; break; }
          fail("expected ',' or ']'");
        }
      }
    } else if (c == '"') {
      v.kind = Json::Str;
      v.s = string();
    } else if (lit("true")) {
      v.kind = Json::Bool;
      v.b = true;
    } else if (lit("false")) {
      v.kind = Json::Bool;
    } else if (lit("null")) {
      v.kind = Json::Null;
    } else {
      const char* start = t_.c_str() + i_;
      char* end = nullptr;
      v.n = std::strtod(start, &end);
      if (end == start) fail("bad value");
      v.kind = Json::Num;
      i_ += (size_t)(end - start);
    }
    --depth_;
    return v;
  }
  std::string string() {
    ++i_;  // opening quote
    std::string out;
    while (i_ < t_.size() && t_[i_] != '"') {
      char c = t_[i_++];
      if (c == '\\') {
        if (i_ >= t_.size()) fail("bad escape");
        char e = t_[i_++];
        switch (e) {
          case 'n': out += '\n'; break;
          case 't': out += '\t'; break;
          case 'r': out += '\r'; break;
          case 'b': out += '\b'; break;
          case 'f': out += '\f'; break;
          case 'u': {
            if (i_ + 4 > t_.size()) fail("bad \\u escape");
            unsigned cp = (unsigned)std::strtoul(t_.substr(i_, 4).c_str(), nullptr, 16);
            i_ += 4;
            if (cp < 0x80) out += (char)cp;
            else out += '?';
            break;
          }
          default: out += e;
        }
      } else {
        out += c;
      }
    }
    if (i_ >= t_.size()) fail("unterminated string");
    ++i_;
    return out;
  }
};

}  // namespace td

// OpenQASM 2.0 reader for the stabilizer subset (host code only): turns a
// circuit text into the library's operation records.
//
// Accepted: the version line, include lines (ignored), qreg and creg
// declarations, the gates id x y z h s sdg cx cy cz swap iswap (and the
// built-in CX) on single qubits or whole registers (broadcast over equal
// sizes), parameterless gate definitions built from accepted gates (expanded
// at each call), measure q -> c (qubit or whole register; outcomes follow in
// program order, the classical target is not recorded), barrier (ignored)
// and // comments. Qubits of several registers are numbered in declaration
// order. Anything else (parameters, reset, if, opaque, U) is rejected with
// its line number.
#include <cctype>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/sq.h"

namespace {

struct Tok {
  enum Kind { ID, INT, STR, SYM, END } kind;
  std::string text;
  int line;
};

struct QasmError {
  std::string msg;
};

[[noreturn]] void die(int line, const std::string &m) { throw QasmError{"line " + std::to_string(line) + ": " + m}; }

std::vector<Tok> tokenize(const char *s, size_t len) {
  std::vector<Tok> out;
  int line = 1;
  size_t i = 0;
  while (i < len) {
    const char c = s[i];
    if (c == '\n') { ++line; ++i; continue; }
    if (isspace((unsigned char)c)) { ++i; continue; }
    if (c == '/' && i + 1 < len && s[i + 1] == '/') {
      while (i < len && s[i] != '\n') ++i;
      continue;
    }
    if (isalpha((unsigned char)c) || c == '_') {
      size_t j = i;
      while (j < len && (isalnum((unsigned char)s[j]) || s[j] == '_')) ++j;
      out.push_back({Tok::ID, std::string(s + i, j - i), line});
      i = j;
      continue;
    }
    if (isdigit((unsigned char)c)) {
      size_t j = i;
      while (j < len && (isdigit((unsigned char)s[j]) || s[j] == '.')) ++j;
      out.push_back({Tok::INT, std::string(s + i, j - i), line});
      i = j;
      continue;
    }
    if (c == '"') {
      size_t j = i + 1;
      while (j < len && s[j] != '"' && s[j] != '\n') ++j;
      if (j >= len || s[j] != '"') die(line, "unterminated string");
      out.push_back({Tok::STR, std::string(s + i + 1, j - i - 1), line});
      i = j + 1;
      continue;
    }
    if (c == '-' && i + 1 < len && s[i + 1] == '>') {
      out.push_back({Tok::SYM, "->", line});
      i += 2;
      continue;
    }
    if (strchr("[](),;{}+-*/^=<>!", c)) {  // arithmetic only reaches the rejection of parameters
      out.push_back({Tok::SYM, std::string(1, c), line});
      ++i;
      continue;
    }
    die(line, std::string("unexpected character '") + c + "'");
  }
  out.push_back({Tok::END, "", line});
  return out;
}

struct Reg {
  uint32_t base, size;
};

// A qubit argument: a register (whole) or one of its qubits.
struct Arg {
  uint32_t base, size;  // size 1 and base = the qubit for an indexed argument
  bool whole;
};

struct GateDef {
  std::vector<std::string> formals;
  std::vector<Tok> body;  // tokens between the braces
  int line;
};

const std::map<std::string, std::pair<uint32_t, int>> &builtins() {
  // name -> (op type, qubit count)
  static const std::map<std::string, std::pair<uint32_t, int>> m = {
      {"id", {SQ_I, 1}},   {"x", {SQ_X, 1}},    {"y", {SQ_Y, 1}},       {"z", {SQ_Z, 1}},
      {"h", {SQ_H, 1}},    {"s", {SQ_S, 1}},    {"sdg", {SQ_SDG, 1}},   {"cx", {SQ_CX, 2}},
      {"CX", {SQ_CX, 2}},  {"cy", {SQ_CY, 2}},  {"cz", {SQ_CZ, 2}},     {"swap", {SQ_SWAP, 2}},
      {"iswap", {SQ_ISWAP, 2}}};
  return m;
}

class Parser {
 public:
  explicit Parser(std::vector<Tok> t) : t_(std::move(t)) {}
  std::vector<sq_op> ops;
  uint32_t nqubits = 0;

  void run() {
    if (peek().kind == Tok::ID && peek().text == "OPENQASM") {
      next();
      const Tok v = next();
      if (v.kind != Tok::INT || (v.text != "2.0" && v.text != "2")) die(v.line, "only OpenQASM 2.0 is read");
      expect(";");
    }
    while (peek().kind != Tok::END) statement();
  }

 private:
  std::vector<Tok> t_;
  size_t pos_ = 0;
  std::map<std::string, Reg> qregs_, cregs_;
  std::map<std::string, GateDef> defs_;

  const Tok &peek() const { return t_[pos_]; }
  Tok next() {
    Tok k = t_[pos_];
    if (k.kind != Tok::END) ++pos_;
    return k;
  }
  void expect(const char *sym) {
    const Tok k = next();
    if (k.kind != Tok::SYM || k.text != sym) die(k.line, std::string("expected '") + sym + "'");
  }
  std::string ident() {
    const Tok k = next();
    if (k.kind != Tok::ID) die(k.line, "expected a name");
    return k.text;
  }
  uint32_t integer() {
    const Tok k = next();
    if (k.kind != Tok::INT || k.text.find('.') != std::string::npos) die(k.line, "expected an integer");
    if (k.text.size() > 9) die(k.line, "integer too large");
    return (uint32_t)std::stoul(k.text);
  }

  void statement() {
    const Tok k = peek();
    if (k.kind != Tok::ID) die(k.line, "expected a statement");
    const std::string &w = k.text;
    if (w == "include") {
      next();
      if (next().kind != Tok::STR) die(k.line, "expected a file name");
      expect(";");
    } else if (w == "qreg" || w == "creg") {
      next();
      const std::string name = ident();
      expect("[");
      const uint32_t size = integer();
      expect("]");
      expect(";");
      if (size == 0) die(k.line, "empty register");
      if (qregs_.count(name) || cregs_.count(name)) die(k.line, "register '" + name + "' declared twice");
      if (w == "qreg") {
        if ((uint64_t)nqubits + size > SQ_MAX_QUBITS) die(k.line, "too many qubits");
        qregs_[name] = Reg{nqubits, size};
        nqubits += size;
      } else {
        cregs_[name] = Reg{0, size};
      }
    } else if (w == "gate") {
      next();
      gate_def(k.line);
    } else if (w == "measure") {
      next();
      const Arg q = qarg();
      expect("->");
      const Arg c = carg();
      expect(";");
      if (q.whole != c.whole || q.size != c.size) die(k.line, "measure: qubit and bit arguments differ in size");
      for (uint32_t i = 0; i < q.size; ++i) ops.push_back(sq_op{SQ_MEASURE, q.base + i, 0});
    } else if (w == "barrier") {
      next();
      qarg();
      while (peek().kind == Tok::SYM && peek().text == ",") {
        next();
        qarg();
      }
      expect(";");
    } else if (w == "reset" || w == "if" || w == "opaque" || w == "U") {
      die(k.line, "'" + w + "' is not supported (stabilizer gates and Z measurements only)");
    } else {
      next();
      call(w, k.line);
    }
  }

  Arg qarg() {
    const Tok k = peek();
    const std::string name = ident();
    auto it = qregs_.find(name);
    if (it == qregs_.end()) die(k.line, "unknown quantum register '" + name + "'");
    return index_of(it->second, k.line);
  }
  Arg carg() {
    const Tok k = peek();
    const std::string name = ident();
    auto it = cregs_.find(name);
    if (it == cregs_.end()) die(k.line, "unknown classical register '" + name + "'");
    return index_of(it->second, k.line);
  }
  Arg index_of(const Reg &r, int line) {
    if (peek().kind == Tok::SYM && peek().text == "[") {
      next();
      const uint32_t i = integer();
      expect("]");
      if (i >= r.size) die(line, "index " + std::to_string(i) + " out of range");
      return Arg{r.base + i, 1, false};
    }
    return Arg{r.base, r.size, true};
  }

  void gate_def(int line) {
    const std::string name = ident();
    if (builtins().count(name)) {
      // a definition of a gate the reader knows (as Qiskit writes for iswap): keep the built-in
      skip_braced_body(line);
      return;
    }
    if (peek().kind == Tok::SYM && peek().text == "(") die(line, "gate '" + name + "': parameters are not supported");
    GateDef d;
    d.line = line;
    d.formals.push_back(ident());
    while (peek().kind == Tok::SYM && peek().text == ",") {
      next();
      d.formals.push_back(ident());
    }
    expect("{");
    int depth = 1;
    while (true) {
      const Tok k = next();
      if (k.kind == Tok::END) die(line, "gate '" + name + "': missing '}'");
      if (k.kind == Tok::SYM && k.text == "{") ++depth;
      if (k.kind == Tok::SYM && k.text == "}" && --depth == 0) break;
      d.body.push_back(k);
    }
    d.body.push_back({Tok::END, "", line});
    defs_[name] = d;
  }

  void skip_braced_body(int line) {
    while (!(peek().kind == Tok::SYM && peek().text == "{")) {
      if (peek().kind == Tok::END) die(line, "gate definition without a body");
      next();
    }
    int depth = 0;
    do {
      const Tok k = next();
      if (k.kind == Tok::END) die(line, "missing '}'");
      if (k.kind == Tok::SYM && k.text == "{") ++depth;
      if (k.kind == Tok::SYM && k.text == "}") --depth;
    } while (depth > 0);
  }

  // A gate call at top level: arguments are registers or indexed qubits.
  void call(const std::string &name, int line) {
    if (peek().kind == Tok::SYM && peek().text == "(") die(line, "gate '" + name + "': parameters are not supported");
    std::vector<Arg> args{qarg()};
    while (peek().kind == Tok::SYM && peek().text == ",") {
      next();
      args.push_back(qarg());
    }
    expect(";");
    uint32_t width = 1;
    for (const Arg &a : args)
      if (a.whole) {
        if (width != 1 && a.size != width) die(line, "registers of different sizes in one call");
        width = a.size;
      }
    for (uint32_t i = 0; i < width; ++i) {
      std::vector<uint32_t> q;
      for (const Arg &a : args) q.push_back(a.whole ? a.base + i : a.base);
      apply(name, q, line, 0);
    }
  }

  void apply(const std::string &name, const std::vector<uint32_t> &q, int line, int depth) {
    if (depth > 32) die(line, "gate definitions nest too deeply");
    auto b = builtins().find(name);
    if (b != builtins().end()) {
      if ((int)q.size() != b->second.second) die(line, "gate '" + name + "' takes " +
                                                 std::to_string(b->second.second) + " qubit(s)");
      if (q.size() == 2 && q[0] == q[1]) die(line, "gate '" + name + "' on the same qubit twice");
      if (b->second.first != SQ_I) ops.push_back(sq_op{b->second.first, q[0], q.size() == 2 ? q[1] : 0u});
      return;
    }
    auto d = defs_.find(name);
    if (d == defs_.end()) die(line, "unknown gate '" + name + "'");
    const GateDef &g = d->second;
    if (g.formals.size() != q.size()) die(line, "gate '" + name + "' takes " + std::to_string(g.formals.size()) +
                                                " qubit(s)");
    // the body: calls on the formal arguments
    size_t i = 0;
    while (g.body[i].kind != Tok::END) {
      const Tok &nm = g.body[i++];
      if (nm.kind != Tok::ID) die(nm.line, "expected a gate call in the body of '" + name + "'");
      if (nm.text == "barrier") {
        while (g.body[i].kind != Tok::END && !(g.body[i].kind == Tok::SYM && g.body[i].text == ";")) ++i;
        if (g.body[i].kind == Tok::END) die(nm.line, "missing ';'");
        ++i;
        continue;
      }
      std::vector<uint32_t> sub;
      while (true) {
        const Tok &a = g.body[i++];
        if (a.kind != Tok::ID) die(a.line, "expected a formal argument");
        size_t f = 0;
        while (f < g.formals.size() && g.formals[f] != a.text) ++f;
        if (f == g.formals.size()) die(a.line, "'" + a.text + "' is not an argument of '" + name + "'");
        sub.push_back(q[f]);
        const Tok &sep = g.body[i++];
        if (sep.kind == Tok::SYM && sep.text == ",") continue;
        if (sep.kind == Tok::SYM && sep.text == ";") break;
        die(sep.line, "expected ',' or ';'");
      }
      apply(nm.text, sub, nm.line, depth + 1);
    }
  }
};

thread_local std::string q_err;

}  // namespace

// The message of the last failed sq_qasm_parse is also what sq_last_error
// reports; the runtime owns that slot, so it is set through this hook.
void sq_set_error_message(const char *msg);

extern "C" sq_status sq_qasm_parse(const char *text, size_t len, sq_op *host_ops, uint64_t cap, uint64_t *count,
                                   uint32_t *n) {
  if (!text || !count || !n || (cap && !host_ops)) {
    sq_set_error_message("sq_qasm_parse: NULL argument");
    return SQ_EINVAL;
  }
  try {
    Parser p(tokenize(text, len));
    p.run();
    *count = p.ops.size();
    *n = p.nqubits;
    for (uint64_t i = 0; i < p.ops.size() && i < cap; ++i) host_ops[i] = p.ops[i];
    return SQ_OK;
  } catch (const QasmError &e) {
    q_err = "sq_qasm_parse: " + e.msg;
    sq_set_error_message(q_err.c_str());
    return SQ_EINVAL;
  } catch (const std::exception &e) {
    q_err = std::string("sq_qasm_parse: ") + e.what();
    sq_set_error_message(q_err.c_str());
    return SQ_ENOMEM;
  }
}

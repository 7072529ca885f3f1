// Circuit text parser (host).  Format: "qubits <n>", optional "grid <r> <c>",
// then "<layer> <gate> <q> [<q2>]" per line; '#' starts a comment.  Gates: h,
// sx, sy, t, cz, and the controlled gates cx and cy (control first).
#include <cctype>
#include <cstdlib>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "qs_internal.h"

namespace qs {

static bool parse_int(const std::string& s, long long& v) {
  if (s.empty()) return false;
  char* end = nullptr;
  v = std::strtoll(s.c_str(), &end, 10);
  return end && *end == '\0';
}

bool parse_circuit(const char* text, size_t len, Circuit& out, std::string& err) {
  Circuit c;
  std::string all(text, len);
  size_t pos = 0;
  int lineno = 0;
  int last_cycle = -1;
  std::set<int> used;  // qubits used in last_cycle
  bool have_n = false;
  while (pos <= all.size()) {
    size_t nl = all.find('\n', pos);
    if (nl == std::string::npos) nl = all.size();
    std::string line = all.substr(pos, nl - pos);
    pos = nl + 1;
    ++lineno;
    size_t hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::vector<std::string> tok;
    {
      size_t i = 0;
      while (i < line.size()) {
        while (i < line.size() && std::isspace((unsigned char)line[i])) ++i;
        size_t j = i;
        while (j < line.size() && !std::isspace((unsigned char)line[j])) ++j;
        if (j > i) tok.push_back(line.substr(i, j - i));
        i = j;
      }
    }
    if (tok.empty()) {
      if (nl == all.size()) break;
      continue;
    }
    auto fail = [&](const std::string& m) {
      err = "line " + std::to_string(lineno) + ": " + m;
      return false;
    };
    if (tok[0] == "qubits") {
      long long v;
      if (tok.size() != 2 || !parse_int(tok[1], v) || v < 1 || v > 64)
        return fail("'qubits' needs a count in 1..64");
      if (have_n) return fail("'qubits' given twice");
      c.n = (int)v;
      have_n = true;
      continue;
    }
    if (tok[0] == "grid") continue;
    if (!have_n) return fail("gate before 'qubits'");
    if (tok.size() < 3) return fail("expected '<layer> <gate> <qubits>'");
    long long t;
    if (!parse_int(tok[0], t) || t < 0 || t > (1LL << 30)) return fail("bad layer number");
    if ((int)t < last_cycle) return fail("layers must not decrease");
    if ((int)t != last_cycle) used.clear();
    last_cycle = (int)t;
    Gate g{(int)t, G_H, -1, -1};
    const std::string& name = tok[1];
    int want = 1;
    if (name == "h") g.kind = G_H;
    else if (name == "sx") g.kind = G_SX;
    else if (name == "sy") g.kind = G_SY;
    else if (name == "t") g.kind = G_T;
    else if (name == "cz") { g.kind = G_CZ; want = 2; }
    else if (name == "cx" || name == "cy") { g.kind = G_CZ; want = 2; }
    else return fail("unknown gate '" + name + "'");
    if ((int)tok.size() != 2 + want) return fail("gate '" + name + "' takes " + std::to_string(want) + " qubit(s)");
    int qv[2] = {-1, -1};
    for (int i = 0; i < want; ++i) {
      long long q;
      if (!parse_int(tok[2 + i], q) || q < 0 || q >= c.n) return fail("qubit out of range");
      qv[i] = (int)q;
      if (used.count(qv[i])) return fail("qubit used twice in one layer");
      used.insert(qv[i]);
    }
    g.q0 = qv[0];
    g.q1 = qv[1];
    if (name == "cx" || name == "cy") {
      // (I x V) CZ (I x V^dagger) on (control q0, target q1), in time order
      const bool y = name == "cy";
      Gate h{(int)t, G_H, qv[1], -1};
      h.aux = true;
      Gate sdg{(int)t, G_T, qv[1], -1, 6, true}, s2{(int)t, G_T, qv[1], -1, 2, true};
      if (y) c.gates.push_back(sdg);
      c.gates.push_back(h);
      c.gates.push_back(g);
      c.gates.push_back(h);
      if (y) c.gates.push_back(s2);
    } else {
      c.gates.push_back(g);
    }
    if (nl == all.size()) break;
  }
  if (!have_n) {
    err = "missing 'qubits' line";
    return false;
  }
  out = std::move(c);
  return true;
}

}  // namespace qs

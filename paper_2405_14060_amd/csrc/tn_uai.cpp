// Model, evidence and query files in the UAI inference-competition text
// format (the format of the problem sets the paper benchmarks on), and
// read-back of a loaded network.
//
// Model file: a preamble word (MARKOV or BAYES), the number of variables,
// their domain sizes, the number of functions, each function's scope (its
// size, then its variable ids), then each function's table (its entry count,
// then the entries, row-major over the scope with the last variable
// fastest).  Tokens are separated by any white space, so tables may span
// lines.  A BAYES file's functions are conditional probability tables whose
// scope ends with the child; the layout is the same, so both kinds load as a
// product of factor tables.
// Evidence file: either "n v_1 x_1 ... v_n x_n" (one evidence set) or
// "m" followed by m such sets.  Query file: "n q_1 ... q_n".
#include <cctype>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tn_internal.h"

namespace {

struct Tokens {
  std::vector<std::string> t;
  size_t i = 0;
  std::string path;
  bool done() const { return i >= t.size(); }
  const std::string &next(const char *what) {
    if (i >= t.size()) throw TnError(TN_E_INVALID, path + ": file ends where " + what + " was expected");
    return t[i++];
  }
  long long integer(const char *what) {
    const std::string &s = next(what);
    char *end = nullptr;
    errno = 0;
    const long long v = std::strtoll(s.c_str(), &end, 10);
    if (errno || end == s.c_str() || *end)
      throw TnError(TN_E_INVALID, path + ": '" + s + "' is not an integer (" + what + ", token " + std::to_string(i) + ")");
    return v;
  }
  double real(const char *what) {
    const std::string &s = next(what);
    char *end = nullptr;
    errno = 0;
    const double v = std::strtod(s.c_str(), &end);
    if (end == s.c_str() || *end)
      throw TnError(TN_E_INVALID, path + ": '" + s + "' is not a number (" + what + ", token " + std::to_string(i) + ")");
    return v;
  }
};

Tokens read_tokens(const char *path) {
  if (!path) throw TnError(TN_E_INVALID, "NULL path");
  FILE *f = std::fopen(path, "rb");
  if (!f) throw TnError(TN_E_INVALID, std::string("cannot open ") + path);
  Tokens tk;
  tk.path = path;
  std::string cur;
  int c;
  while ((c = std::fgetc(f)) != EOF) {
    if (std::isspace(c)) {
      if (!cur.empty()) tk.t.push_back(std::move(cur)), cur.clear();
    } else {
      cur.push_back((char)c);
    }
  }
  if (!cur.empty()) tk.t.push_back(std::move(cur));
  std::fclose(f);
  return tk;
}

template <class F>
tn_status guard_uai(F &&f) {
  try {
    f();
    return TN_OK;
  } catch (const TnError &e) {
    tn::set_last_error(e.what());
    return e.st;
  } catch (const std::bad_alloc &) {
    tn::set_last_error("host allocation failed");
    return TN_E_NOMEM;
  } catch (const std::exception &e) {
    tn::set_last_error(e.what());
    return TN_E_INVALID;
  }
}

}  // namespace

extern "C" tn_status tn_load_uai(const char *path, tn_net **out) {
  return guard_uai([&] {
    if (!out) throw TnError(TN_E_INVALID, "NULL output");
    Tokens tk = read_tokens(path);
    std::string kind = tk.next("the preamble (MARKOV or BAYES)");
    for (char &ch : kind) ch = (char)std::toupper((unsigned char)ch);
    if (kind != "MARKOV" && kind != "BAYES")
      throw TnError(TN_E_INVALID, tk.path + ": preamble '" + kind + "' is neither MARKOV nor BAYES");
    const long long n = tk.integer("the number of variables");
    if (n < 0 || n > (1 << 24)) throw TnError(TN_E_INVALID, tk.path + ": bad number of variables");
    std::vector<int32_t> card((size_t)n);
    for (long long v = 0; v < n; ++v) {
      const long long c = tk.integer("a domain size");
      if (c < 1 || c > (1 << 20)) throw TnError(TN_E_INVALID, tk.path + ": bad domain size of variable " + std::to_string(v));
      card[(size_t)v] = (int32_t)c;
    }
    const long long nf = tk.integer("the number of functions");
    if (nf < 0 || nf > (1 << 26)) throw TnError(TN_E_INVALID, tk.path + ": bad number of functions");
    std::vector<int64_t> sp((size_t)nf + 1, 0);
    std::vector<int32_t> sv;
    std::vector<double> size_of((size_t)nf, 1.0);
    for (long long f = 0; f < nf; ++f) {
      const long long k = tk.integer("a scope size");
      if (k < 0 || k > 64) throw TnError(TN_E_INVALID, tk.path + ": bad scope size of function " + std::to_string(f));
      for (long long j = 0; j < k; ++j) {
        const long long v = tk.integer("a scope variable");
        if (v < 0 || v >= n) throw TnError(TN_E_INVALID, tk.path + ": scope variable out of range in function " + std::to_string(f));
        sv.push_back((int32_t)v);
        size_of[(size_t)f] *= card[(size_t)v];
      }
      sp[(size_t)f + 1] = (int64_t)sv.size();
    }
    std::vector<double> vals;
    for (long long f = 0; f < nf; ++f) {
      const long long m = tk.integer("a table size");
      if ((double)m != size_of[(size_t)f])
        throw TnError(TN_E_INVALID, tk.path + ": function " + std::to_string(f) + " has " + std::to_string(m) +
                                        " entries, its scope needs " + std::to_string((long long)size_of[(size_t)f]));
      for (long long j = 0; j < m; ++j) vals.push_back(tk.real("a table entry"));
    }
    if (!tk.done()) throw TnError(TN_E_INVALID, tk.path + ": unexpected tokens after the last table");
    const tn_status st = tn_load_network((int32_t)n, card.data(), (int32_t)nf, sp.data(), sv.data(), vals.data(), 0, out);
    if (st != TN_OK) throw TnError(st, tk.path + ": " + std::string(tn_last_error()));
  });
}

extern "C" tn_status tn_read_uai_evidence(const char *path, int32_t n_vars, const int32_t *card, int32_t *evidence,
                                          int32_t cap_rows, int32_t *n_rows) {
  return guard_uai([&] {
    if (n_vars < 0 || (n_vars > 0 && !card) || !n_rows) throw TnError(TN_E_INVALID, "NULL argument");
    Tokens tk = read_tokens(path);
    std::vector<long long> x;
    while (!tk.done()) x.push_back(tk.integer("an integer"));
    if (x.empty()) throw TnError(TN_E_INVALID, tk.path + ": empty evidence file");
    std::vector<std::vector<std::pair<long long, long long>>> sets;
    auto parse_set = [&](size_t &i) {
      if (i >= x.size()) throw TnError(TN_E_INVALID, tk.path + ": evidence set count missing");
      const long long k = x[i++];
      if (k < 0 || i + 2 * (size_t)k > x.size()) throw TnError(TN_E_INVALID, tk.path + ": truncated evidence set");
      std::vector<std::pair<long long, long long>> s;
      for (long long j = 0; j < k; ++j, i += 2) s.push_back({x[i], x[i + 1]});
      sets.push_back(std::move(s));
    };
    if (x[0] >= 0 && x.size() == 1 + 2 * (size_t)x[0]) {  // one set
      size_t i = 0;
      parse_set(i);
    } else {  // a count of sets, then the sets
      size_t i = 1;
      for (long long s = 0; s < x[0]; ++s) parse_set(i);
      if (x[0] < 0 || i != x.size()) throw TnError(TN_E_INVALID, tk.path + ": malformed evidence file");
    }
    *n_rows = (int32_t)sets.size();
    for (size_t r = 0; r < sets.size() && (int32_t)r < cap_rows; ++r) {
      if (!evidence) throw TnError(TN_E_INVALID, "NULL evidence buffer");
      int32_t *row = evidence + r * (size_t)n_vars;
      for (int32_t v = 0; v < n_vars; ++v) row[v] = -1;
      for (auto &pv : sets[r]) {
        if (pv.first < 0 || pv.first >= n_vars) throw TnError(TN_E_INVALID, tk.path + ": evidence variable out of range");
        if (pv.second < 0 || pv.second >= card[pv.first])
          throw TnError(TN_E_INVALID, tk.path + ": evidence value out of range for variable " + std::to_string(pv.first));
        if (row[pv.first] >= 0 && row[pv.first] != pv.second)
          throw TnError(TN_E_INVALID, tk.path + ": variable " + std::to_string(pv.first) + " observed twice");
        row[pv.first] = (int32_t)pv.second;
      }
    }
  });
}

extern "C" tn_status tn_read_uai_query(const char *path, int32_t n_vars, int32_t *vars, int32_t cap, int32_t *n) {
  return guard_uai([&] {
    if (!n) throw TnError(TN_E_INVALID, "NULL argument");
    Tokens tk = read_tokens(path);
    const long long k = tk.integer("the number of query variables");
    if (k < 0 || k > n_vars) throw TnError(TN_E_INVALID, tk.path + ": bad number of query variables");
    std::vector<char> seen((size_t)n_vars, 0);
    *n = (int32_t)k;
    for (long long j = 0; j < k; ++j) {
      const long long v = tk.integer("a query variable");
      if (v < 0 || v >= n_vars) throw TnError(TN_E_INVALID, tk.path + ": query variable out of range");
      if (seen[(size_t)v]) throw TnError(TN_E_INVALID, tk.path + ": query variable listed twice");
      seen[(size_t)v] = 1;
      if (j < cap) {
        if (!vars) throw TnError(TN_E_INVALID, "NULL query buffer");
        vars[j] = (int32_t)v;
      }
    }
    if (!tk.done()) throw TnError(TN_E_INVALID, tk.path + ": unexpected tokens after the query");
  });
}

extern "C" tn_status tn_network_sizes(const tn_net *net, int32_t *n_vars, int32_t *n_factors, int64_t *n_scope,
                                      int64_t *n_values) {
  return guard_uai([&] {
    if (!net) throw TnError(TN_E_INVALID, "NULL network");
    if (n_vars) *n_vars = net->n_vars;
    if (n_factors) *n_factors = (int32_t)net->scope.size();
    if (n_scope) {
      int64_t s = 0;
      for (auto &sc : net->scope) s += (int64_t)sc.size();
      *n_scope = s;
    }
    if (n_values) *n_values = net->n_values;
  });
}

extern "C" tn_status tn_network_get(const tn_net *net, int32_t *card, int64_t *scope_ptr, int32_t *scope_vars,
                                    double *values, int32_t *values_are_log) {
  return guard_uai([&] {
    if (!net) throw TnError(TN_E_INVALID, "NULL network");
    if (card)
      for (int v = 0; v < net->n_vars; ++v) card[v] = net->card[v];
    int64_t o = 0;
    if (scope_ptr) scope_ptr[0] = 0;
    for (size_t f = 0; f < net->scope.size(); ++f) {
      for (int v : net->scope[f]) {
        if (scope_vars) scope_vars[o] = v;
        ++o;
      }
      if (scope_ptr) scope_ptr[f + 1] = o;
    }
    if (values)
      for (size_t f = 0; f < net->vals.size(); ++f)
        std::memcpy(values + net->val_off[f], net->vals[f].data(), net->vals[f].size() * sizeof(double));
    if (values_are_log) *values_are_log = net->is_log ? 1 : 0;
  });
}

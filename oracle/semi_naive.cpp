// Oracle: a plain, slow, single-threaded CPU evaluator of positive Datalog
// over uint32 relations of arity 1..4.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
// call this file; only the tests, the smoke check and the CPU-baseline leg
// of the benchmark use it.  It shares no code with the GPU library: its own
// parser, its own relation store (std::set), its own join loop.
//
// What it computes.  The result of a positive Datalog program is its least
// model: the smallest IDB sets closed under every rule.  Semi-naive
// evaluation (Section 2, "Semi-naive evaluation") reaches exactly that set
// by joining each rule against the tuples found in the previous iteration
// (the delta version) instead of against everything (the full version),
// and by keeping delta and full disjoint (Section 2, the SG example): the
// delta of an iteration is the new tuples minus the full version, and the
// loop stops when every delta is empty (Section 5.1, fixpoint workflow).
//
// Schedule (a reading: the paper does not fix the order of rules inside
// one iteration).  Jacobi: iteration 0 evaluates the rules whose bodies
// hold only EDB atoms; iteration i >= 1 evaluates every rule that has an
// IDB body atom once per IDB atom position t, with atom t ranging over the
// delta of iteration i-1 and every other IDB atom over the full version of
// iteration i-1 (which already includes that delta); only after all rules
// are the deltas formed and merged.  Under this schedule the full version
// after iteration i equals naive evaluation's after i+1 applications of
// the immediate-consequence operator, so the per-iteration delta sizes are
// as well defined as the final sets.
//
// The naive mode (recompute every rule over the full versions each
// iteration) is kept as a second algorithm for cross-checks.
//
// Filters: `x != y` between two body variables (the SG rules, Section 2).
// Wildcard `_` binds nothing.  No constants, negation or aggregates.

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

namespace {

typedef std::array<uint32_t, 4> Tuple;  // unused trailing columns are 0

struct Atom {
  int rel = -1;
  std::vector<int> args;  // variable id, or -1 for the wildcard
};

struct Filter {
  int a, b;  // variable ids: keep the binding only when a != b
};

struct Rule {
  Atom head;
  std::vector<Atom> body;
  std::vector<Filter> filters;
  int nvars = 0;
};

struct Relation {
  std::string name;
  int arity = 0;
  bool edb = false;
  std::set<Tuple> full, delta, fresh;
  // Secondary copies of `full`, one per bound-column mask: each tuple is
  // permuted so the bound columns come first, so that every lookup is a
  // prefix range on an ordered set.
  std::map<int, std::set<Tuple>> index;
  std::vector<uint64_t> delta_counts;
  std::vector<uint64_t> new_counts;  // per iteration: distinct derived tuples, before subtracting full
  // Per-iteration copies of the delta and new sets, kept on request (small inputs only).
  std::vector<std::set<Tuple>> delta_history, new_history;
};

Tuple permute(const Tuple& t, int arity, int mask) {
  Tuple p{0, 0, 0, 0};
  int k = 0;
  for (int c = 0; c < arity; ++c)
    if (mask & (1 << c)) p[k++] = t[c];
  for (int c = 0; c < arity; ++c)
    if (!(mask & (1 << c))) p[k++] = t[c];
  return p;
}

Tuple unpermute(const Tuple& p, int arity, int mask) {
  Tuple t{0, 0, 0, 0};
  int k = 0;
  for (int c = 0; c < arity; ++c)
    if (mask & (1 << c)) t[c] = p[k++];
  for (int c = 0; c < arity; ++c)
    if (!(mask & (1 << c))) t[c] = p[k++];
  return t;
}

// ---------------------------------------------------------------- parser

struct Parser {
  const std::string& s;
  size_t i = 0;
  explicit Parser(const std::string& text) : s(text) {}

  void skip() {
    for (;;) {
      while (i < s.size() && isspace((unsigned char)s[i])) ++i;
      if (i + 1 < s.size() && s[i] == '/' && s[i + 1] == '/') {
        while (i < s.size() && s[i] != '\n') ++i;
      } else if (i < s.size() && s[i] == '#') {
        while (i < s.size() && s[i] != '\n') ++i;
      } else {
        return;
      }
    }
  }
  bool eof() { skip(); return i >= s.size(); }
  bool peek(const char* lit) {
    skip();
    return s.compare(i, strlen(lit), lit) == 0;
  }
  void expect(const char* lit) {
    if (!peek(lit)) throw std::runtime_error(std::string("expected '") + lit + "' at offset " + std::to_string(i));
    i += strlen(lit);
  }
  std::string ident() {
    skip();
    size_t b = i;
    while (i < s.size() && (isalnum((unsigned char)s[i]) || s[i] == '_')) ++i;
    if (b == i) throw std::runtime_error("expected an identifier at offset " + std::to_string(i));
    return s.substr(b, i - b);
  }
};

}  // namespace

struct OracleEngine {
  std::vector<Relation> rels;
  std::vector<Rule> rules;
  std::string err;
  int iterations = 0;
  double seconds = 0.0;
  int plant = 0;  // test hook: plants one known mistake (see or_run)
  int max_iterations = 1 << 30;
  bool keep_history = false;

  int find(const std::string& n) const {
    for (size_t k = 0; k < rels.size(); ++k)
      if (rels[k].name == n) return (int)k;
    return -1;
  }

  Atom parse_atom(Parser& p, std::map<std::string, int>& vars, int& nvars) {
    Atom a;
    std::string name = p.ident();
    a.rel = find(name);
    if (a.rel < 0) throw std::runtime_error("undeclared relation " + name);
    p.expect("(");
    for (;;) {
      std::string v = p.ident();
      if (v == "_") {
        a.args.push_back(-1);
      } else {
        if (!(isalpha((unsigned char)v[0]))) throw std::runtime_error("bad variable " + v);
        auto it = vars.find(v);
        if (it == vars.end()) it = vars.emplace(v, nvars++).first;
        a.args.push_back(it->second);
      }
      if (p.peek(",")) { p.expect(","); continue; }
      p.expect(")");
      break;
    }
    if ((int)a.args.size() != rels[a.rel].arity)
      throw std::runtime_error("arity mismatch for " + name);
    return a;
  }

  void parse(const std::string& text) {
    Parser p(text);
    std::vector<Rule> out;
    while (!p.eof()) {
      Rule r;
      std::map<std::string, int> vars;
      r.head = parse_atom(p, vars, r.nvars);
      if (rels[r.head.rel].edb) throw std::runtime_error("rule head is an EDB relation");
      p.expect(":-");
      for (;;) {
        // a filter `x != y` or an atom
        size_t save = p.i;
        std::string id = p.ident();
        if (p.peek("!=")) {
          p.expect("!=");
          std::string id2 = p.ident();
          auto a = vars.find(id), b = vars.find(id2);
          if (a == vars.end() || b == vars.end())
            throw std::runtime_error("filter variable not bound by an earlier atom");
          r.filters.push_back({a->second, b->second});
        } else {
          p.i = save;
          r.body.push_back(parse_atom(p, vars, r.nvars));
        }
        if (p.peek(",")) { p.expect(","); continue; }
        p.expect(".");
        break;
      }
      // range restriction: every head variable appears in the body
      for (int v : r.head.args) {
        if (v < 0) throw std::runtime_error("wildcard in rule head");
        bool found = false;
        for (auto& a : r.body)
          for (int w : a.args) found |= (w == v);
        if (!found) throw std::runtime_error("head variable not bound in the body");
      }
      out.push_back(r);
    }
    rules.insert(rules.end(), out.begin(), out.end());
  }

  const std::set<Tuple>& full_index(int rel, int mask) {
    Relation& R = rels[rel];
    auto it = R.index.find(mask);
    if (it != R.index.end()) return it->second;
    std::set<Tuple>& ix = R.index[mask];
    for (const Tuple& t : R.full) ix.insert(permute(t, R.arity, mask));
    return ix;
  }

  // Depth-first enumeration of the body bindings in `order`.
  void enumerate(const Rule& r, const std::vector<int>& order, const std::vector<int>& use_delta,
                 size_t k, std::vector<uint32_t>& val, std::vector<char>& bound) {
    if (k == order.size()) {
      for (const Filter& f : r.filters) {
        bool differ = val[f.a] != val[f.b];
        if (plant == 3) differ = !differ;  // planted: filter sense inverted
        if (!differ) return;
      }
      Tuple h{0, 0, 0, 0};
      const Relation& H = rels[r.head.rel];
      for (int c = 0; c < H.arity; ++c) h[c] = val[r.head.args[c]];
      rels[r.head.rel].fresh.insert(h);
      return;
    }
    const Atom& a = r.body[order[k]];
    Relation& R = rels[a.rel];
    const int arity = R.arity;
    auto try_tuple = [&](const Tuple& t) {
      int newly[4];
      int nn = 0;
      bool ok = true;
      for (int c = 0; c < arity && ok; ++c) {
        int v = a.args[c];
        if (v < 0) continue;
        if (bound[v]) {
          ok = (val[v] == t[c]);
        } else {
          val[v] = t[c];
          bound[v] = 1;
          newly[nn++] = v;
        }
      }
      if (ok) enumerate(r, order, use_delta, k + 1, val, bound);
      for (int q = 0; q < nn; ++q) bound[newly[q]] = 0;
    };
    if (use_delta[order[k]]) {
      for (const Tuple& t : R.delta) try_tuple(t);
      return;
    }
    int mask = 0;
    for (int c = 0; c < arity; ++c)
      if (a.args[c] >= 0 && bound[a.args[c]]) mask |= 1 << c;
    if (mask == 0) {
      for (const Tuple& t : R.full) try_tuple(t);
      return;
    }
    const std::set<Tuple>& ix = full_index(a.rel, mask);
    Tuple lo{0, 0, 0, 0};
    int nb = 0;
    for (int c = 0; c < arity; ++c)
      if (mask & (1 << c)) lo[nb++] = val[a.args[c]];
    for (auto it = ix.lower_bound(lo); it != ix.end(); ++it) {
      bool same = true;
      for (int q = 0; q < nb; ++q) same &= ((*it)[q] == lo[q]);
      if (!same) break;
      if (plant == 5) {  // planted: the last tuple of every range is skipped
        auto nx = std::next(it);
        bool last = nx == ix.end();
        for (int q = 0; q < nb && !last; ++q) last |= ((*nx)[q] != lo[q]);
        if (last) break;
      }
      try_tuple(unpermute(*it, arity, mask));
    }
  }

  // Body order: the delta atom first (or atom 0), then repeatedly the first
  // remaining atom that shares a bound variable (else the first remaining).
  std::vector<int> order_for(const Rule& r, int first) {
    std::vector<int> order{first};
    std::vector<char> used(r.body.size(), 0);
    used[first] = 1;
    std::vector<char> b(r.nvars, 0);
    for (int v : r.body[first].args) if (v >= 0) b[v] = 1;
    while (order.size() < r.body.size()) {
      int pick = -1;
      for (size_t j = 0; j < r.body.size() && pick < 0; ++j) {
        if (used[j]) continue;
        for (int v : r.body[j].args) if (v >= 0 && b[v]) { pick = (int)j; break; }
      }
      if (pick < 0)
        for (size_t j = 0; j < r.body.size(); ++j) if (!used[j]) { pick = (int)j; break; }
      used[pick] = 1;
      order.push_back(pick);
      for (int v : r.body[pick].args) if (v >= 0) b[v] = 1;
    }
    return order;
  }

  void eval_rule(const Rule& r, const std::vector<int>& use_delta, int first) {
    std::vector<uint32_t> val(r.nvars, 0);
    std::vector<char> bound(r.nvars, 0);
    enumerate(r, order_for(r, first), use_delta, 0, val, bound);
  }

  // Forms every delta from the fresh tuples and merges it into full.
  // Returns the total delta size.
  uint64_t close_iteration() {
    uint64_t total = 0;
    for (Relation& R : rels) {
      if (R.edb) continue;
      R.delta.clear();
      R.new_counts.push_back(R.fresh.size());
      if (keep_history) R.new_history.push_back(R.fresh);
      for (const Tuple& t : R.fresh)
        if (plant == 6 || !R.full.count(t)) R.delta.insert(t);  // planted 6: no subtraction
      R.fresh.clear();
      for (const Tuple& t : R.delta) {
        R.full.insert(t);
        for (auto& ix : R.index) ix.second.insert(permute(t, R.arity, ix.first));
      }
      R.delta_counts.push_back(R.delta.size());
      if (keep_history) R.delta_history.push_back(R.delta);
      total += R.delta.size();
    }
    return total;
  }

  bool is_edb_only(const Rule& r) const {
    for (const Atom& a : r.body) if (!rels[a.rel].edb) return false;
    return true;
  }

  static void reset(Relation& R) {
    R.full.clear();
    R.delta.clear();
    R.fresh.clear();
    R.index.clear();
    R.delta_counts.clear();
    R.new_counts.clear();
    R.delta_history.clear();
    R.new_history.clear();
  }

  void check_cap() {
    if (iterations > max_iterations) throw std::runtime_error("iteration cap exceeded");
  }

  void run_semi_naive() {
    for (Relation& R : rels) if (!R.edb) reset(R);
    iterations = 0;
    // iteration 0: rules over EDB atoms only
    for (const Rule& r : rules)
      if (is_edb_only(r)) eval_rule(r, std::vector<int>(r.body.size(), 0), 0);
    uint64_t d = close_iteration();
    iterations = 1;
    while (d != 0) {
      for (const Rule& r : rules) {
        if (is_edb_only(r)) continue;
        int seen = 0;
        for (size_t t = 0; t < r.body.size(); ++t) {
          if (rels[r.body[t].rel].edb) continue;
          if (plant == 1 && seen++ > 0) break;  // planted: only the first delta variant
          if (rels[r.body[t].rel].delta.empty()) continue;
          std::vector<int> use(r.body.size(), 0);
          use[t] = 1;
          eval_rule(r, use, (int)t);
          if (plant == 4) close_iteration_partial(r.head.rel);  // planted: Gauss-Seidel
        }
      }
      d = close_iteration();
      ++iterations;
      check_cap();
    }
  }

  // Planted mistake 4 only: merges one relation's fresh tuples early.
  void close_iteration_partial(int rel) {
    Relation& R = rels[rel];
    for (const Tuple& t : R.fresh) {
      if (R.full.insert(t).second)
        for (auto& ix : R.index) ix.second.insert(permute(t, R.arity, ix.first));
    }
    R.fresh.clear();
  }

  void run_naive() {
    for (Relation& R : rels) if (!R.edb) reset(R);
    iterations = 0;
    uint64_t d;
    do {
      for (const Rule& r : rules) eval_rule(r, std::vector<int>(r.body.size(), 0), 0);
      d = close_iteration();
      ++iterations;
      check_cap();
    } while (d != 0);
  }
};

// ------------------------------------------------------------------ C ABI

extern "C" {

OracleEngine* or_create() { return new OracleEngine(); }
void or_destroy(OracleEngine* e) { delete e; }
const char* or_error(OracleEngine* e) { return e->err.c_str(); }

int or_declare(OracleEngine* e, const char* name, int arity, int is_edb) {
  if (arity < 1 || arity > 4) { e->err = "arity must be 1..4"; return -1; }
  if (e->find(name) >= 0) { e->err = "relation declared twice"; return -1; }
  Relation R;
  R.name = name;
  R.arity = arity;
  R.edb = is_edb != 0;
  e->rels.push_back(R);
  return 0;
}

int or_load(OracleEngine* e, const char* name, const uint32_t* rows, uint64_t n) {
  int k = e->find(name);
  if (k < 0 || !e->rels[k].edb) { e->err = "no such EDB relation"; return -1; }
  Relation& R = e->rels[k];
  for (uint64_t i = 0; i < n; ++i) {
    Tuple t{0, 0, 0, 0};
    for (int c = 0; c < R.arity; ++c) t[c] = rows[i * R.arity + c];
    R.full.insert(t);
  }
  R.index.clear();
  return 0;
}

int or_program(OracleEngine* e, const char* text) {
  try {
    e->parse(text);
  } catch (const std::exception& x) {
    e->err = x.what();
    return -1;
  }
  return 0;
}

// mode 0: semi-naive (Jacobi); mode 1: naive.  `plant` is a test hook that
// plants one known mistake so the tests can show that the pins catch it:
// 1 drops every delta variant but the first, 3 inverts filters, 4 merges
// early (Gauss-Seidel), 5 skips the last tuple of each index range, 6 keeps
// tuples already in full in the delta.  0 is the correct evaluator.
int or_run(OracleEngine* e, int mode, int plant, int max_iterations, int keep_history) {
  e->plant = plant;
  e->max_iterations = max_iterations > 0 ? max_iterations : (1 << 30);
  e->keep_history = keep_history != 0;
  auto t0 = std::chrono::steady_clock::now();
  try {
    if (mode == 0) e->run_semi_naive();
    else e->run_naive();
  } catch (const std::exception& x) {
    e->err = x.what();
    return -1;
  }
  e->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return 0;
}

int or_iterations(OracleEngine* e) { return e->iterations; }
double or_seconds(OracleEngine* e) { return e->seconds; }

int64_t or_count(OracleEngine* e, const char* name) {
  int k = e->find(name);
  if (k < 0) return -1;
  return (int64_t)e->rels[k].full.size();
}

int or_new_counts(OracleEngine* e, const char* name, uint64_t* out, int cap) {
  int k = e->find(name);
  if (k < 0) return -1;
  Relation& R = e->rels[k];
  int n = (int)R.new_counts.size();
  for (int i = 0; i < n && i < cap; ++i) out[i] = R.new_counts[i];
  return n;
}

// which = 0: the delta of iteration `iter`; 1: its new set.  Needs history.
int64_t or_history(OracleEngine* e, const char* name, int which, int iter, uint32_t* rows,
                   uint64_t cap) {
  int k = e->find(name);
  if (k < 0) return -1;
  Relation& R = e->rels[k];
  const auto& hist = which == 0 ? R.delta_history : R.new_history;
  if (iter < 0 || iter >= (int)hist.size()) return -1;
  const std::set<Tuple>& S = hist[iter];
  if (cap < S.size()) return -2;
  uint64_t i = 0;
  for (const Tuple& t : S) {
    for (int c = 0; c < R.arity; ++c) rows[i * R.arity + c] = t[c];
    ++i;
  }
  return (int64_t)S.size();
}

// Row-major, lexicographic in declared column order.
int or_fetch(OracleEngine* e, const char* name, uint32_t* rows, uint64_t cap) {
  int k = e->find(name);
  if (k < 0) return -1;
  Relation& R = e->rels[k];
  if (cap < R.full.size()) return -2;
  uint64_t i = 0;
  for (const Tuple& t : R.full) {
    for (int c = 0; c < R.arity; ++c) rows[i * R.arity + c] = t[c];
    ++i;
  }
  return 0;
}

int or_delta_counts(OracleEngine* e, const char* name, uint64_t* out, int cap) {
  int k = e->find(name);
  if (k < 0) return -1;
  Relation& R = e->rels[k];
  int n = (int)R.delta_counts.size();
  for (int i = 0; i < n && i < cap; ++i) out[i] = R.delta_counts[i];
  return n;
}

// ---------------------------------------------------------------------------
// Independent checker for Reach: per-source breadth-first search (textbook).
// hist[d] receives the number of pairs (s, t) whose shortest directed path
// has exactly d >= 1 edges (a pair (s, s) counts when s lies on a cycle,
// with d the length of its shortest cycle).  Returns the number of pairs.
// Pairs at distance d are exactly the Reach tuples first derived in
// iteration d-1 of the Jacobi schedule.

int64_t or_reach_bfs(uint32_t n_nodes, const uint32_t* edges, uint64_t m, uint64_t* hist,
                     int hist_cap, int threads) {
  std::vector<uint64_t> off(n_nodes + 1, 0);
  for (uint64_t i = 0; i < m; ++i) {
    if (edges[2 * i] >= n_nodes || edges[2 * i + 1] >= n_nodes) return -1;
    off[edges[2 * i] + 1]++;
  }
  for (uint32_t v = 0; v < n_nodes; ++v) off[v + 1] += off[v];
  std::vector<uint32_t> adj(m);
  {
    std::vector<uint64_t> cur(off.begin(), off.end() - 1);
    for (uint64_t i = 0; i < m; ++i) adj[cur[edges[2 * i]]++] = edges[2 * i + 1];
  }
  if (threads < 1) threads = 1;
  std::atomic<uint32_t> next{0};
  std::vector<std::vector<uint64_t>> local(threads, std::vector<uint64_t>(hist_cap, 0));
  std::atomic<bool> overflow{false};
  auto work = [&](int tid) {
    std::vector<uint32_t> dist(n_nodes, UINT32_MAX), queue(n_nodes);
    std::vector<uint64_t>& h = local[tid];
    for (;;) {
      uint32_t s = next.fetch_add(1);
      if (s >= n_nodes) break;
      size_t qh = 0, qt = 0;
      dist[s] = 0;
      queue[qt++] = s;
      uint32_t self = UINT32_MAX;
      while (qh < qt) {
        uint32_t u = queue[qh++];
        for (uint64_t k = off[u]; k < off[u + 1]; ++k) {
          uint32_t v = adj[k];
          if (v == s && self == UINT32_MAX) self = dist[u] + 1;
          if (dist[v] == UINT32_MAX) {
            dist[v] = dist[u] + 1;
            queue[qt++] = v;
          }
        }
      }
      for (size_t q = 1; q < qt; ++q) {
        uint32_t d = dist[queue[q]];
        if ((int)d < hist_cap) h[d]++;
        else overflow = true;
      }
      if (self != UINT32_MAX) {
        if ((int)self < hist_cap) h[self]++;
        else overflow = true;
      }
      for (size_t q = 0; q < qt; ++q) dist[queue[q]] = UINT32_MAX;
    }
  };
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) pool.emplace_back(work, t);
  for (auto& t : pool) t.join();
  if (overflow) return -2;
  int64_t total = 0;
  for (int d = 0; d < hist_cap; ++d) {
    hist[d] = 0;
    for (int t = 0; t < threads; ++t) hist[d] += local[t][d];
    total += (int64_t)hist[d];
  }
  return total;
}

// Sorted targets reachable from `source` by one or more edges.
int64_t or_reach_from(uint32_t n_nodes, const uint32_t* edges, uint64_t m, uint32_t source,
                      uint32_t* out, uint64_t cap) {
  if (source >= n_nodes) return -1;
  std::vector<std::vector<uint32_t>> adj(n_nodes);
  for (uint64_t i = 0; i < m; ++i) {
    if (edges[2 * i] >= n_nodes || edges[2 * i + 1] >= n_nodes) return -1;
    adj[edges[2 * i]].push_back(edges[2 * i + 1]);
  }
  std::vector<char> seen(n_nodes, 0);
  std::vector<uint32_t> stack;
  for (uint32_t v : adj[source]) if (!seen[v]) { seen[v] = 1; stack.push_back(v); }
  while (!stack.empty()) {
    uint32_t u = stack.back();
    stack.pop_back();
    for (uint32_t v : adj[u]) if (!seen[v]) { seen[v] = 1; stack.push_back(v); }
  }
  uint64_t n = 0;
  for (uint32_t v = 0; v < n_nodes; ++v)
    if (seen[v]) {
      if (n < cap) out[n] = v;
      ++n;
    }
  return (int64_t)n;
}

}  // extern "C"

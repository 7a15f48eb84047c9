// Host mechanism compiler: validation, phase x instance expansion, state ids, Jacobian
// pattern, fill-reducing order, symbolic LU fill and level-scheduled tables.
//
// The paper's Processes declare at initialization the Jacobian elements they contribute to
// (so the solver may use a sparse Jacobian) and receive ids for species and Jacobian
// elements for use during solving (table of Process functions: get_used_jacobian_elements,
// update_ids). Processes on an aerosol phase apply to every instance of the phase
// (Sect. 2.2.3). The linear solver is a sparse direct LU (Sect. 2.4.1, KLU); here its
// pattern, fill and elimination schedule are fixed once per mechanism so every cell of
// every call shares them.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <set>
#include <sstream>
#include <cstdint>
#include <cstring>

#include "mech.hpp"

namespace camp {

namespace {

constexpr double kAvogadro = 6.02214076e23;
constexpr int kWaveLanes = 64;

bool finite(double v) { return std::isfinite(v); }

struct Bits {
  int n = 0, words = 0;
  std::vector<uint64_t> w;
  void init(int n_, int rows) {
    n = n_;
    words = (n + 63) / 64;
    w.assign((size_t)words * rows, 0);
  }
  uint64_t* row(int r) { return w.data() + (size_t)r * words; }
  bool get(int r, int c) const { return (w[(size_t)r * words + c / 64] >> (c % 64)) & 1u; }
  void set(int r, int c) { w[(size_t)r * words + c / 64] |= (uint64_t)1 << (c % 64); }
};

// Minimum degree on the symmetrized pattern (elimination-graph model). With level_aware,
// the next vertex is chosen among those whose degree is within `slack` of the minimum as the
// one with the shallowest elimination depth (1 + the depth of the deepest eliminated
// neighbour), then the lowest degree: the sparse triangular solves and the LU then have
// fewer dependency levels, usually for about the same fill. Ties go to the lowest index, so
// the order is deterministic.
std::vector<int> minimum_degree(int n, const std::vector<std::pair<int, int>>& edges,
                                bool level_aware = false, int slack = 0) {
  std::vector<std::set<int>> adj(n);
  for (auto& e : edges)
    if (e.first != e.second) {
      adj[e.first].insert(e.second);
      adj[e.second].insert(e.first);
    }
  std::vector<char> alive(n, 1);
  std::vector<int> depth(n, 0);
  std::vector<int> order;
  order.reserve(n);
  for (int step = 0; step < n; ++step) {
    size_t md = SIZE_MAX;
    for (int v = 0; v < n; ++v)
      if (alive[v]) md = std::min(md, adj[v].size());
    int best = -1;
    for (int v = 0; v < n; ++v) {
      if (!alive[v] || adj[v].size() > md + (level_aware ? (size_t)slack : 0)) continue;
      if (best < 0) {
        best = v;
      } else if (level_aware) {
        if (depth[v] < depth[best] || (depth[v] == depth[best] && adj[v].size() < adj[best].size()))
          best = v;
      } else if (adj[v].size() < adj[best].size()) {
        best = v;
      }
    }
    order.push_back(best);
    alive[best] = 0;
    std::vector<int> nb(adj[best].begin(), adj[best].end());
    for (int a : nb) {
      adj[a].erase(best);
      for (int b : nb)
        if (b != a) adj[a].insert(b);
      depth[a] = std::max(depth[a], depth[best] + 1);
    }
    adj[best].clear();
  }
  return order;
}

// Symbolic fill of the (unsymmetric) pattern in elimination order `order` (row k of the
// result: columns of the filled row of the k-th eliminated variable).
Bits symbolic_fill(int n, const std::vector<std::pair<int, int>>& edges, const std::vector<int>& order) {
  std::vector<int> ip(n);
  for (int t = 0; t < n; ++t) ip[order[t]] = t;
  Bits F;
  F.init(n, n);
  for (auto& e : edges) F.set(ip[e.first], ip[e.second]);
  for (int k = 0; k < n; ++k) {
    // rows i > k with (i, k): OR row k's entries right of k into row i
    for (int i = k + 1; i < n; ++i) {
      if (!F.get(i, k)) continue;
      uint64_t* ri = F.row(i);
      const uint64_t* rk = F.row(k);
      for (int w = 0; w < F.words; ++w) {
        uint64_t m = rk[w];
        int lo = w * 64;
        if (lo + 63 <= k) continue;
        if (lo <= k) m &= ~((k - lo == 63) ? ~0ull : ((1ull << (k - lo + 1)) - 1));
        ri[w] |= m;
      }
    }
  }
  return F;
}

// Cost of an elimination order for the level-scheduled device work: filled entries, and the
// dependency levels of the forward sweep, the backward sweep and the Crout LU.
struct OrderCost {
  long long nnz = 0;
  int fwd = 0, bwd = 0, lu = 0;
  // per Newton iteration both sweeps run; an LU serves several iterations
  long long weight() const { return 7LL * (fwd + bwd) + lu; }
};

OrderCost order_cost(int n, const Bits& F) {
  OrderCost c;
  std::vector<int> lf(n, 0), lb(n, 0);
  for (int t = 0; t < n; ++t)
    for (int j = 0; j < t; ++j)
      if (F.get(t, j)) lf[t] = std::max(lf[t], lf[j] + 1);
  for (int t = n - 1; t >= 0; --t)
    for (int j = t + 1; j < n; ++j)
      if (F.get(t, j)) lb[t] = std::max(lb[t], lb[j] + 1);
  // Crout: entry (i, j) is computed from (i, k), (k, j) for k < min(i, j) and, below the
  // diagonal, the pivot (j, j)
  std::vector<int> L((size_t)n * n, 0);
  for (int m = 0; m < n; ++m) {
    auto entry = [&](int i, int j) {
      const int mn = std::min(i, j);
      int l = 0;
      bool task = i > j;
      for (int k = 0; k < mn; ++k)
        if (F.get(i, k) && F.get(k, j)) {
          l = std::max(l, std::max(L[(size_t)i * n + k], L[(size_t)k * n + j]));
          task = true;
        }
      if (i > j) l = std::max(l, L[(size_t)j * n + j]);
      L[(size_t)i * n + j] = task ? l + 1 : 0;
      c.lu = std::max(c.lu, L[(size_t)i * n + j]);
    };
    for (int j = m; j < n; ++j)
      if (F.get(m, j)) entry(m, j);
    for (int i = m + 1; i < n; ++i)
      if (F.get(i, m)) entry(i, m);
  }
  for (int t = 0; t < n; ++t) {
    c.fwd = std::max(c.fwd, lf[t]);
    c.bwd = std::max(c.bwd, lb[t]);
    for (int j = 0; j < n; ++j) c.nnz += F.get(t, j);
  }
  return c;
}

// Elimination order: plain minimum degree and level-aware variants; the one with the fewest
// weighted dependency levels whose fill stays within 10 % of the plain order's.
std::vector<int> choose_order(int n, const std::vector<std::pair<int, int>>& edges) {
  std::vector<int> best = minimum_degree(n, edges);
  const OrderCost base = order_cost(n, symbolic_fill(n, edges, best));
  OrderCost bc = base;
  for (int slack = 0; slack <= 3; ++slack) {
    std::vector<int> o = minimum_degree(n, edges, true, slack);
    const OrderCost c = order_cost(n, symbolic_fill(n, edges, o));
    if (c.nnz * 10 > base.nnz * 11) continue;
    if (c.weight() < bc.weight() || (c.weight() == bc.weight() && c.nnz < bc.nnz)) {
      bc = c;
      best = std::move(o);
    }
  }
  return best;
}

// Dependency levels of the wavefront engine's factor and solve when the last K positions
// form a dense tail handled through the inverse of their Schur complement (see StageBlock):
// forward levels over the head rows and the tail rows' head columns, backward levels over
// the head rows, Crout levels where tail entries sum over head pivots only.
struct TailCost {
  int fwd = 0, bwd = 0, lu = 0;
  // Measured on the fused kernel (cycles of one group): a sweep level costs about half an
  // LU level, a Gauss-Jordan step about as much as an LU level, and one factorization serves
  // about seven Newton iterations; weights per factorization interval: sweep level 7, LU level
  // 3, Gauss-Jordan step 3, plus one sweep level for the product with the inverse.
  long long weight(int K) const { return 7LL * (fwd + bwd + (K ? 1 : 0)) + 3LL * lu + (K ? 3LL * (K + 1) : 0); }
};

TailCost tail_cost(int n, const Bits& F, int K) {
  const int s = n - K;
  TailCost c;
  std::vector<int> lf(n, 0), lb(n, 0);
  for (int t = 0; t < n; ++t)
    for (int j = 0; j < t; ++j)
      if (F.get(t, j) && (t < s || j < s)) lf[t] = std::max(lf[t], lf[j] + 1);
  for (int t = s - 1; t >= 0; --t)
    for (int j = t + 1; j < n; ++j)
      if (F.get(t, j)) lb[t] = std::max(lb[t], lb[j] + 1);
  std::vector<int> L((size_t)n * n, 0);
  for (int m = 0; m < n; ++m) {
    auto entry = [&](int i, int j) {
      const bool tail = i >= s && j >= s;
      const int mn = tail ? s : std::min(i, j);
      int l = 0;
      bool task = i > j && !tail;
      for (int k = 0; k < mn; ++k)
        if (F.get(i, k) && F.get(k, j)) {
          l = std::max(l, std::max(L[(size_t)i * n + k], L[(size_t)k * n + j]));
          task = true;
        }
      if (i > j && !tail) l = std::max(l, L[(size_t)j * n + j]);
      L[(size_t)i * n + j] = task ? l + 1 : 0;
      c.lu = std::max(c.lu, L[(size_t)i * n + j]);
    };
    for (int j = m; j < n; ++j)
      if (F.get(m, j)) entry(m, j);
    for (int i = m + 1; i < n; ++i)
      if (F.get(i, m)) entry(i, m);
  }
  for (int t = 0; t < n; ++t) {
    c.fwd = std::max(c.fwd, lf[t]);
    c.bwd = std::max(c.bwd, lb[t]);
  }
  return c;
}

// Pattern F with its trailing K x K block made dense.
Bits with_dense_tail(const Bits& F, int n, int K) {
  Bits G = F;
  for (int i = n - K; i < n; ++i)
    for (int j = n - K; j < n; ++j) G.set(i, j);
  return G;
}

// Size of the dense tail: the K (0 or 2..k_max) of least TailCost::weight whose dense block
// adds at most 6 % to the stored entries. Ties keep the smaller block.
int choose_tail(int n, const Bits& F, long long nnz, int k_max) {
  int best_k = 0;
  long long best_w = tail_cost(n, F, 0).weight(0);
  for (int K = 2; K <= std::min(k_max, n - 1); ++K) {
    long long have = 0;
    for (int i = n - K; i < n; ++i)
      for (int j = n - K; j < n; ++j) have += F.get(i, j);
    if (((long long)K * K - have) * 100 > 6 * nnz) continue;
    const long long w = tail_cost(n, with_dense_tail(F, n, K), K).weight(K);
    if (w < best_w) {
      best_w = w;
      best_k = K;
    }
  }
  return best_k;
}

}  // namespace

int max_tail(int wave_lists) {
  // rows per wavefront ceil(K / W), split over max(1, 64 / K) lane groups, at most
  // kTailPerLane per lane; K <= 64 (one column per lane)
  auto fits = [&](int K) {
    const int rows = (K + wave_lists - 1) / wave_lists, groups = std::max(1, kWaveLanes / K);
    return (rows + groups - 1) / groups <= (wave_lists == 1 ? kTailPerLaneOneWave : kTailPerLane);
  };
  int k = 0;
  while (k + 1 <= kWaveLanes && fits(k + 1)) ++k;
  return k;
}

std::string compile_mechanism(const camp_reaction* rxns, int n_rxn, const camp_species* sp,
                              int n_sp, const camp_phase* ph, int n_ph, Compiled& C) {
  std::ostringstream err;
  if (n_sp <= 0 || !sp) return "mechanism has no species";
  if (n_rxn < 0 || (n_rxn > 0 && !rxns)) return "bad reaction array";
  if (n_ph < 0 || (n_ph > 0 && !ph)) return "bad phase array";

  // ---- species and phases ----
  std::vector<int> gas_state(n_sp, -1), sp_phase(n_sp), pos_in_phase(n_sp, -1);
  int n_gas = 0;
  for (int s = 0; s < n_sp; ++s) {
    sp_phase[s] = sp[s].phase;
    if (sp[s].phase < -1 || sp[s].phase >= n_ph) {
      err << "species " << s << " has invalid phase " << sp[s].phase;
      return err.str();
    }
    if (sp[s].phase < 0) gas_state[s] = n_gas++;
  }
  std::vector<int> phase_first_inst(n_ph), phase_base(n_ph);
  int n_inst = 0, pos = n_gas;
  for (int p = 0; p < n_ph; ++p) {
    const camp_phase& q = ph[p];
    if (q.n_species < 1 || !q.species) {
      err << "phase " << p << " has no species";
      return err.str();
    }
    if (q.n_instances < 1) {
      err << "phase " << p << " has no instances";
      return err.str();
    }
    if (!(q.density_kg_m3 > 0) || !finite(q.density_kg_m3) || !(q.mw_absorber_kg_mol > 0) ||
        !finite(q.mw_absorber_kg_mol)) {
      err << "phase " << p << " needs positive finite density and absorber molar mass";
      return err.str();
    }
    for (int k = 0; k < q.n_species; ++k) {
      int s = q.species[k];
      if (s < 0 || s >= n_sp || sp[s].phase != p || pos_in_phase[s] >= 0) {
        err << "phase " << p << " lists species " << s << " that does not belong to it";
        return err.str();
      }
      pos_in_phase[s] = k;
    }
    phase_first_inst[p] = n_inst;
    phase_base[p] = pos;
    for (int i = 0; i < q.n_instances; ++i) {
      C.inst_phase.push_back(p);
      C.inst_base.push_back(pos);
      pos += q.n_species;
    }
    n_inst += q.n_instances;
  }
  for (int s = 0; s < n_sp; ++s)
    if (sp[s].phase >= 0 && pos_in_phase[s] < 0) {
      err << "species " << s << " is not listed by its phase";
      return err.str();
    }
  const int N = pos;
  C.n_state = N;
  C.n_gas = n_gas;
  C.n_inst = n_inst;

  auto cond_state = [&](int p, int inst_local, int s) {
    return phase_base[p] + inst_local * ph[p].n_species + pos_in_phase[s];
  };

  // ---- expansion ----
  struct X {
    int nr, np;
    int react[3], prod[3];
    double yld[3];
    // Parameters (Sect. 2.2.2) over the state indices pspec: kParamRaoult divides the rate by
    // kc[pconst] + sum of y; kParamRadius evaluates the transfer rate at the radius grown by
    // sum of pw * y (entries pnum, pcore, ppath; accommodation palpha)
    int pflags = 0;
    int pconst = -1, pnum = -1, pcore = -1, ppath = -1;
    double palpha = 0.0;
    std::vector<int> pspec;
    std::vector<double> pw;
  };
  std::vector<X> xs;
  std::vector<RateSpec> rs;
  int n_ext = 0;
  for (int r = 0; r < n_rxn; ++r) {
    const camp_reaction& q = rxns[r];
    for (int v = 0; v < 10; ++v)
      if (!finite(q.p[v])) {
        err << "reaction " << r << " has a non-finite parameter";
        return err.str();
      }
    if (q.n_react < 0 || q.n_react > 3 || q.n_prod < 0 || q.n_prod > 3) {
      err << "reaction " << r << ": n_react and n_prod must be within 0..3";
      return err.str();
    }
    for (int k = 0; k < q.n_react; ++k)
      if (q.react[k] < 0 || q.react[k] >= n_sp) {
        err << "reaction " << r << ": reactant id out of range";
        return err.str();
      }
    for (int k = 0; k < q.n_prod; ++k) {
      if (q.prod[k] < 0 || q.prod[k] >= n_sp) {
        err << "reaction " << r << ": product id out of range";
        return err.str();
      }
      if (!finite(q.yield[k]) || q.yield[k] < 0) {
        err << "reaction " << r << ": yields must be finite and >= 0";
        return err.str();
      }
      for (int k2 = 0; k2 < k; ++k2)
        if (q.prod[k2] == q.prod[k]) {
          err << "reaction " << r << ": duplicate product";
          return err.str();
        }
    }
    const int t = q.type;
    auto base_spec = [&](int kind) {
      RateSpec s{};
      s.kind = kind;
      s.ext = -1;
      s.inst = -1;
      return s;
    };
    const bool gas_special = t == CAMP_RXN_TROE || t == CAMP_RXN_CUSTOM_H2O2 ||
                             t == CAMP_RXN_CUSTOM_OH_HNO3 || t == CAMP_RXN_WENNBERG_TUNNELING;
    if (t == CAMP_RXN_ARRHENIUS || t == CAMP_RXN_PHOTOLYSIS || t == CAMP_RXN_EMISSION ||
        t == CAMP_RXN_FIRST_ORDER_LOSS || gas_special) {
      for (int k = 0; k < q.n_react; ++k)
        if (gas_state[q.react[k]] < 0) {
          err << "reaction " << r << ": gas-phase process with a condensed reactant";
          return err.str();
        }
      for (int k = 0; k < q.n_prod; ++k)
        if (gas_state[q.prod[k]] < 0) {
          err << "reaction " << r << ": gas-phase process with a condensed product";
          return err.str();
        }
      RateSpec s;
      if (gas_special) {
        // positive pre-exponential factors where the form divides by them; Fc, N > 0
        bool ok = true;
        if (t == CAMP_RXN_TROE)
          ok = q.p[0] >= 0 && q.p[3] > 0 && q.p[6] > 0 && q.p[7] > 0;
        else if (t == CAMP_RXN_CUSTOM_H2O2)
          ok = q.p[0] >= 0 && q.p[3] >= 0;
        else if (t == CAMP_RXN_CUSTOM_OH_HNO3)
          ok = q.p[0] >= 0 && q.p[3] > 0 && q.p[6] >= 0;
        else
          ok = q.p[0] >= 0;
        if (!ok) {
          err << "reaction " << r << ": invalid rate parameters for its type";
          return err.str();
        }
        s = base_spec(t == CAMP_RXN_TROE ? KR_TROE
                      : t == CAMP_RXN_CUSTOM_H2O2 ? KR_H2O2
                      : t == CAMP_RXN_CUSTOM_OH_HNO3 ? KR_OHHNO3 : KR_TUNNEL);
        for (int v = 0; v < 9; ++v) s.v[v] = q.p[v];
        s.v[9] = std::pow(kAvogadro * 1.0e-6, q.n_react - 1);
      } else if (t == CAMP_RXN_ARRHENIUS) {
        if (q.p[0] < 0 || (q.p[2] != 0.0 && !(q.p[3] > 0))) {
          err << "reaction " << r << ": Arrhenius needs A >= 0 and D > 0 when B != 0";
          return err.str();
        }
        s = base_spec(KR_ARRHENIUS);
        s.v[0] = q.p[0] * std::pow(kAvogadro * 1.0e-6, q.n_react - 1);
        s.v[1] = q.p[1];
        s.v[2] = q.p[2];
        s.v[3] = q.p[3];
        s.v[4] = q.p[4];
      } else {
        if (q.p[0] < 0) {
          err << "reaction " << r << ": negative rate";
          return err.str();
        }
        if (t == CAMP_RXN_PHOTOLYSIS && q.n_react != 1) {
          err << "reaction " << r << ": photolysis needs exactly one reactant";
          return err.str();
        }
        if (t == CAMP_RXN_EMISSION && (q.n_react != 0 || q.n_prod != 1)) {
          err << "reaction " << r << ": emission needs 0 reactants and 1 product";
          return err.str();
        }
        if (t == CAMP_RXN_FIRST_ORDER_LOSS && (q.n_react != 1 || q.n_prod != 0)) {
          err << "reaction " << r << ": first-order loss needs 1 reactant and 0 products";
          return err.str();
        }
        s = base_spec(t == CAMP_RXN_PHOTOLYSIS ? KR_PHOTOLYSIS
                                                : t == CAMP_RXN_EMISSION ? KR_EMISSION : KR_LOSS);
        s.v[0] = q.p[0];
        s.v[1] = q.p[1];
        s.ext = n_ext++;
      }
      X x{};
      x.nr = q.n_react;
      x.np = q.n_prod;
      for (int k = 0; k < q.n_react; ++k) x.react[k] = gas_state[q.react[k]];
      for (int k = 0; k < q.n_prod; ++k) {
        x.prod[k] = gas_state[q.prod[k]];
        x.yld[k] = q.yield[k];
      }
      s.nr = x.nr;
      xs.push_back(x);
      rs.push_back(s);
    } else if (t == CAMP_RXN_CONDENSED_ARRHENIUS) {
      const int p = q.phase;
      if (p < 0 || p >= n_ph) {
        err << "reaction " << r << ": condensed-phase process needs a valid phase";
        return err.str();
      }
      for (int k = 0; k < q.n_react; ++k)
        if (sp_phase[q.react[k]] != p) {
          err << "reaction " << r << ": reactant not in the reaction's phase";
          return err.str();
        }
      for (int k = 0; k < q.n_prod; ++k)
        if (sp_phase[q.prod[k]] != p) {
          err << "reaction " << r << ": product not in the reaction's phase";
          return err.str();
        }
      if (q.p[0] < 0 || (q.p[2] != 0.0 && !(q.p[3] > 0))) {
        err << "reaction " << r << ": Arrhenius needs A >= 0 and D > 0 when B != 0";
        return err.str();
      }
      for (int i = 0; i < ph[p].n_instances; ++i) {
        RateSpec s = base_spec(KR_CONDENSED);
        s.inst = phase_first_inst[p] + i;
        for (int v = 0; v < 6; ++v) s.v[v] = q.p[v];
        s.v[6] = ph[p].density_kg_m3;
        s.nr = q.n_react;
        X x{};
        x.nr = q.n_react;
        x.np = q.n_prod;
        for (int k = 0; k < q.n_react; ++k) x.react[k] = cond_state(p, i, q.react[k]);
        for (int k = 0; k < q.n_prod; ++k) {
          x.prod[k] = cond_state(p, i, q.prod[k]);
          x.yld[k] = q.yield[k];
        }
        xs.push_back(x);
        rs.push_back(s);
      }
    } else if (t == CAMP_RXN_AQUEOUS_REVERSIBLE) {
      const int p = q.phase;
      if (p < 0 || p >= n_ph) {
        err << "reaction " << r << ": aqueous reversible reaction needs a valid phase";
        return err.str();
      }
      for (int k = 0; k < q.n_react; ++k)
        if (sp_phase[q.react[k]] != p) {
          err << "reaction " << r << ": reactant not in the reaction's phase";
          return err.str();
        }
      for (int k = 0; k < q.n_prod; ++k)
        if (sp_phase[q.prod[k]] != p || q.yield[k] != 1.0) {
          err << "reaction " << r << ": reversible products must be in the phase with yield 1";
          return err.str();
        }
      if (q.n_react < 1 || q.n_prod < 1 || q.p[0] < 0 || q.p[2] < 0) {
        err << "reaction " << r << ": reversible reaction needs reactants, products, A >= 0, k_r >= 0";
        return err.str();
      }
      // the reverse direction: products -> reactants, repeated reactants as yields
      int rv_prod[3], rv_n = 0;
      double rv_yld[3];
      for (int k = 0; k < q.n_react; ++k) {
        int f = -1;
        for (int m = 0; m < rv_n; ++m)
          if (rv_prod[m] == q.react[k]) f = m;
        if (f < 0) {
          rv_prod[rv_n] = q.react[k];
          rv_yld[rv_n++] = 1.0;
        } else {
          rv_yld[f] += 1.0;
        }
      }
      for (int i = 0; i < ph[p].n_instances; ++i)
        for (int dir = 0; dir < 2; ++dir) {
          RateSpec s = base_spec(dir == 0 ? KR_AQREV_FWD : KR_AQREV_REV);
          s.inst = phase_first_inst[p] + i;
          s.v[0] = q.p[0];
          s.v[1] = q.p[1];
          s.v[2] = q.p[2];
          s.v[3] = ph[p].density_kg_m3;
          X x{};
          if (dir == 0) {
            x.nr = q.n_react;
            x.np = q.n_prod;
            for (int k = 0; k < q.n_react; ++k) x.react[k] = cond_state(p, i, q.react[k]);
            for (int k = 0; k < q.n_prod; ++k) {
              x.prod[k] = cond_state(p, i, q.prod[k]);
              x.yld[k] = 1.0;
            }
          } else {
            x.nr = q.n_prod;
            x.np = rv_n;
            for (int k = 0; k < q.n_prod; ++k) x.react[k] = cond_state(p, i, q.prod[k]);
            for (int k = 0; k < rv_n; ++k) {
              x.prod[k] = cond_state(p, i, rv_prod[k]);
              x.yld[k] = rv_yld[k];
            }
          }
          s.nr = x.nr;
          xs.push_back(x);
          rs.push_back(s);
        }
    } else if (t == CAMP_RXN_HENRY_TRANSFER || t == CAMP_RXN_SIMPOL_TRANSFER) {
      const int p = q.phase;
      if (p < 0 || p >= n_ph) {
        err << "reaction " << r << ": transfer process needs a valid phase";
        return err.str();
      }
      if (q.n_react != 1 || q.n_prod != 1 || gas_state[q.react[0]] < 0 ||
          sp_phase[q.prod[0]] != p) {
        err << "reaction " << r << ": transfer needs one gas-phase reactant and one product "
                                   "in the reaction's phase";
        return err.str();
      }
      const camp_species& g = sp[q.react[0]];
      if (!(g.mw_kg_mol > 0) || !(g.diff_m2_s > 0) || !(g.accom > 0) || !finite(g.mw_kg_mol) ||
          !finite(g.diff_m2_s) || !finite(g.accom)) {
        err << "reaction " << r << ": gas partner needs positive MW, diffusion and accommodation";
        return err.str();
      }
      if (t == CAMP_RXN_HENRY_TRANSFER && !(q.p[0] > 0)) {
        err << "reaction " << r << ": Henry constant must be positive";
        return err.str();
      }
      const bool henry = t == CAMP_RXN_HENRY_TRANSFER;
      const bool raoult = !henry && q.p[4] != 0.0;
      const bool grows = ph[p].radius_from_state != 0;
      if (grows && henry) {
        err << "reaction " << r << ": Henry transfer into a phase whose radius follows the state "
                                   "is not supported";
        return err.str();
      }
      if (grows)
        for (int m = 0; m < ph[p].n_species; ++m) {
          const double mw = sp[ph[p].species[m]].mw_kg_mol;
          if (!(mw > 0) || !finite(mw)) {
            err << "reaction " << r << ": species of a phase whose radius follows the state need a "
                                       "positive molecular weight";
            return err.str();
          }
        }
      if (!henry && q.p[4] != 0.0 && q.p[4] != 1.0) {
        err << "reaction " << r << ": SIMPOL full-Raoult flag p[4] must be 0 or 1";
        return err.str();
      }
      if (raoult && !(ph[p].mw_absorber_kg_mol > 0)) {
        err << "reaction " << r << ": full-Raoult SIMPOL needs a positive absorber molecular weight";
        return err.str();
      }
      for (int i = 0; i < ph[p].n_instances; ++i) {
        // entries pushed after the two directions: [absorber], [number, core volume, path]
        const int after = (int)xs.size() + 2;
        const int absorber = raoult ? after : -1;
        const int geo = after + (raoult ? 1 : 0);
        for (int dir = 0; dir < 2; ++dir) {
          RateSpec s = base_spec(henry ? (dir == 0 ? KR_HENRY_COND : KR_HENRY_EVAP)
                                       : (dir == 0 ? KR_SIMPOL_COND
                                                   : (raoult ? KR_SIMPOL_EVAP_RAOULT : KR_SIMPOL_EVAP)));
          s.inst = phase_first_inst[p] + i;
          s.v[0] = g.diff_m2_s;
          s.v[1] = g.mw_kg_mol;
          s.v[2] = g.accom;
          s.v[3] = ph[p].density_kg_m3;
          s.v[4] = ph[p].mw_absorber_kg_mol;
          for (int v = 0; v < 4; ++v) s.v[5 + v] = q.p[v];
          s.nr = 1;
          X x{};
          x.nr = 1;
          x.np = 1;
          int gs = gas_state[q.react[0]], as = cond_state(p, i, q.prod[0]);
          x.react[0] = dir == 0 ? gs : as;
          x.prod[0] = dir == 0 ? as : gs;
          x.yld[0] = 1.0;
          if ((raoult && dir == 1) || grows)
            for (int m = 0; m < ph[p].n_species; ++m)
              x.pspec.push_back(cond_state(p, i, ph[p].species[m]));
          if (raoult && dir == 1) {
            // total condensed amount of the instance: the absorber entry plus every species
            x.pflags |= kParamRaoult;
            x.pconst = absorber;
          }
          if (grows) {
            x.pflags |= kParamRadius;
            x.pnum = geo;
            x.pcore = geo + 1;
            x.ppath = geo + 2;
            x.palpha = g.accom;
            for (int m = 0; m < ph[p].n_species; ++m)
              x.pw.push_back(sp[ph[p].species[m]].mw_kg_mol / ph[p].density_kg_m3);
          }
          xs.push_back(x);
          rs.push_back(s);
        }
        auto carrier = [&](int kind) {
          RateSpec s = base_spec(kind);
          s.inst = phase_first_inst[p] + i;
          s.v[0] = g.diff_m2_s;
          s.v[1] = g.mw_kg_mol;
          s.v[3] = ph[p].density_kg_m3;
          s.v[4] = ph[p].mw_absorber_kg_mol;
          s.nr = 0;
          xs.push_back(X{});
          rs.push_back(s);
        };
        if (raoult) carrier(KR_ABSORBER);
        if (grows) {
          carrier(KR_NUMBER);
          carrier(KR_CORE_VOLUME);
          carrier(KR_MEAN_PATH);
        }
      }
    } else {
      err << "reaction " << r << ": unknown type " << t;
      return err.str();
    }
  }
  const int R = (int)xs.size();
  C.n_rxn = R;
  C.n_ext = n_ext;

  // ---- net stoichiometry and the Jacobian pattern (user order) ----
  // S[i][k] kept sparse: per reaction the distinct members with their net coefficient.
  std::vector<std::vector<std::pair<int, double>>> members(R);
  std::vector<std::pair<int, int>> edges;
  for (int k = 0; k < R; ++k) {
    const X& x = xs[k];
    std::vector<std::pair<int, double>> m;
    auto add = [&](int i, double c) {
      for (auto& e : m)
        if (e.first == i) {
          e.second += c;
          return;
        }
      m.push_back({i, c});
    };
    for (int o = 0; o < x.nr; ++o) add(x.react[o], -1.0);
    for (int o = 0; o < x.np; ++o) add(x.prod[o], x.yld[o]);
    members[k] = m;
    for (int o = 0; o < x.nr; ++o)
      for (auto& e : m) edges.push_back({e.first, x.react[o]});   // (row i, col j)
    for (int j : x.pspec)
      for (auto& e : m) edges.push_back({e.first, j});
  }
  for (int i = 0; i < N; ++i) edges.push_back({i, i});

  // ---- elimination order and symbolic fill ----
  C.perm = choose_order(N, edges);
  C.iperm.assign(N, 0);
  for (int t = 0; t < N; ++t) C.iperm[C.perm[t]] = t;

  Bits F0;
  F0.init(N, N);
  for (auto& e : edges) F0.set(C.iperm[e.first], C.iperm[e.second]);
  Bits F = symbolic_fill(N, edges, C.perm);
  {
    long long nnz = 0, n_part = 0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) nnz += F.get(i, j);
    for (const X& x : xs) n_part += x.nr + n_param_partials(x.pflags);
    // Gauss-Jordan keeps 4K doubles in the partials / rates scratch of a cell
    const int scratch_k = (int)(std::max<long long>(n_part, (long long)xs.size()) / 4);
    C.nnz_lu = (int)nnz;
    C.tail_k = choose_tail(N, F, nnz, std::min(max_tail(4), scratch_k));
    if (C.tail_k > 0) F = with_dense_tail(F, N, C.tail_k);
  }

  // ---- CSR of the filled pattern ----
  C.row_ptr.assign(N + 1, 0);
  C.diag.assign(N, -1);
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j)
      if (F.get(i, j)) {
        if (i == j) C.diag[i] = (int)C.col.size();
        C.col.push_back(j);
        C.pattern0.push_back(F0.get(i, j) ? 1 : 0);
      }
    C.row_ptr[i + 1] = (int)C.col.size();
  }
  C.nnz = (int)C.col.size();
  C.nnz0 = 0;
  for (char c : C.pattern0) C.nnz0 += c;
  auto slot = [&](int i, int j) -> int {
    auto b = C.col.begin() + C.row_ptr[i], e = C.col.begin() + C.row_ptr[i + 1];
    auto it = std::lower_bound(b, e, j);
    return (it != e && *it == j) ? (int)(it - C.col.begin()) : -1;
  };

  // ---- device reaction tables (elimination positions) ----
  C.rate = rs;
  C.rx_react.assign((size_t)R * 3, -1);
  C.rx_nr.assign(R, 0);
  C.rx_pofs.assign(R + 1, 0);
  for (int k = 0; k < R; ++k) {
    C.rx_nr[k] = xs[k].nr;
    for (int o = 0; o < xs[k].nr; ++o) C.rx_react[3 * k + o] = C.iperm[xs[k].react[o]];
    // each Parameter adds one partial after the reactant occurrences: -r / p for the 1/p
    // factor (equal for every j of the set), r dln(psi)/dr / (4 pi N_p r^2) for the radius
    // (times w_j in the Jacobian contributions)
    C.rx_pofs[k + 1] = C.rx_pofs[k] + xs[k].nr + n_param_partials(xs[k].pflags);
  }
  C.n_partials = C.rx_pofs[R];
  C.param_ptr.assign(1, 0);
  C.param.clear();
  C.param_w.clear();
  for (int k = 0; k < R; ++k) {
    const X& x = xs[k];
    if (!x.pflags) continue;
    const int rec[kParamHead] = {k, x.pflags, x.pconst, x.pnum, x.pcore, x.ppath};
    for (int v : rec) {
      C.param.push_back(v);
      C.param_w.push_back(0.0);
    }
    C.param_w[C.param_w.size() - kParamHead + 1] = x.palpha;
    for (size_t j = 0; j < x.pspec.size(); ++j) {
      C.param.push_back(C.iperm[x.pspec[j]]);
      C.param_w.push_back(x.pw.empty() ? 0.0 : x.pw[j]);
    }
    C.param_ptr.push_back((int)C.param.size());
  }

  // forcing terms by species (elimination position), reactions ascending
  {
    std::vector<std::vector<std::pair<int, double>>> by(N);
    for (int k = 0; k < R; ++k)
      for (auto& e : members[k])
        if (e.second != 0.0) by[C.iperm[e.first]].push_back({k, e.second});
    C.term_ptr.assign(N + 1, 0);
    for (int t = 0; t < N; ++t) {
      for (auto& e : by[t]) {
        C.term_rxn.push_back(e.first);
        C.term_coef.push_back(e.second);
      }
      C.term_ptr[t + 1] = (int)C.term_rxn.size();
    }
  }
  // Jacobian contributions by slot: J[i][j] += S[i][k] * partial(k, o) for react[k][o] == j
  {
    std::vector<std::vector<std::pair<int, double>>> by(C.nnz);
    for (int k = 0; k < R; ++k)
      for (int o = 0; o < xs[k].nr; ++o) {
        int j = C.iperm[xs[k].react[o]];
        for (auto& e : members[k]) {
          if (e.second == 0.0) continue;
          int s = slot(C.iperm[e.first], j);
          by[s].push_back({C.rx_pofs[k] + o, e.second});
        }
      }
    for (int k = 0; k < R; ++k) {
      int part = C.rx_pofs[k] + xs[k].nr;
      for (int flag : {kParamRaoult, kParamRadius}) {
        if (!(xs[k].pflags & flag)) continue;
        for (size_t jj = 0; jj < xs[k].pspec.size(); ++jj) {
          const int j = C.iperm[xs[k].pspec[jj]];
          const double w = flag == kParamRadius ? xs[k].pw[jj] : 1.0;
          for (auto& e : members[k]) {
            if (e.second == 0.0) continue;
            by[slot(C.iperm[e.first], j)].push_back({part, e.second * w});
          }
        }
        ++part;
      }
    }
    C.jc_ptr.assign(C.nnz + 1, 0);
    for (int s = 0; s < C.nnz; ++s) {
      for (auto& e : by[s]) {
        C.jc_part.push_back(e.first);
        C.jc_coef.push_back(e.second);
      }
      C.jc_ptr[s + 1] = (int)C.jc_part.size();
    }
  }

  // ---- Crout LU tasks: one per computed entry, in dependency levels ----
  // U entry (i <= j): u_ij = m_ij - sum_{k < i} l_ik u_kj
  // L entry (i >  j): l_ij = (m_ij - sum_{k < j} l_ik u_kj) / u_jj
  {
    std::vector<int> level(C.nnz, 0);
    struct Pending {
      Task t;
      int level;
      std::vector<std::pair<int, int>> pairs;
    };
    std::vector<Pending> pend;
    auto make = [&](int i, int j) {
      int s = slot(i, j);
      int m = std::min(i, j);
      Pending p;
      p.t.dst = s;
      p.t.diag = (i > j) ? C.diag[j] : -1;
      int lv = 0;
      for (int q = C.row_ptr[i]; q < C.row_ptr[i + 1] && C.col[q] < m; ++q) {
        int k = C.col[q];
        int skj = slot(k, j);
        if (skj < 0) continue;
        p.pairs.push_back({q, skj});
        lv = std::max(lv, std::max(level[q], level[skj]));
      }
      if (p.t.diag >= 0) lv = std::max(lv, level[p.t.diag]);
      if (p.pairs.empty() && p.t.diag < 0) return;   // value is final as given
      level[s] = lv + 1;
      p.level = lv + 1;
      pend.push_back(std::move(p));
    };
    for (int m = 0; m < N; ++m) {
      for (int q = C.row_ptr[m]; q < C.row_ptr[m + 1]; ++q)
        if (C.col[q] >= m) make(m, C.col[q]);
      for (int i = m + 1; i < N; ++i)
        if (slot(i, m) >= 0) make(i, m);
    }
    int L = 0;
    for (auto& p : pend) L = std::max(L, p.level);
    std::stable_sort(pend.begin(), pend.end(),
                     [](const Pending& a, const Pending& b) { return a.level < b.level; });
    C.lu_level_ptr.assign(L + 1, 0);
    for (auto& p : pend) {
      Task t = p.t;
      t.pbeg = (int)C.lu_pa.size();
      for (auto& pr : p.pairs) {
        C.lu_pa.push_back(pr.first);
        C.lu_pb.push_back(pr.second);
      }
      t.pend = (int)C.lu_pa.size();
      C.lu_tasks.push_back(t);
      C.lu_level_ptr[p.level]++;   // count, prefix-summed below (levels start at 1)
    }
    // level_ptr[l] .. level_ptr[l+1] for l = 0..L-1 holds level l+1
    std::vector<int> cnt(C.lu_level_ptr);
    C.lu_level_ptr.assign(L + 1, 0);
    for (int l = 1; l <= L; ++l) C.lu_level_ptr[l] = C.lu_level_ptr[l - 1] + cnt[l];
    C.lu_pairs = (long long)C.lu_pa.size();
  }

  // ---- triangular solves ----
  {
    // forward, unit lower: x_t -= sum_{k < t} l_tk x_k
    std::vector<int> lv(N, 0);
    std::vector<std::pair<int, Task>> tk;
    std::vector<std::vector<std::pair<int, int>>> prs;
    for (int t = 0; t < N; ++t) {
      Task T{t, -1, 0, 0};
      std::vector<std::pair<int, int>> pp;
      int l = 0;
      for (int q = C.row_ptr[t]; q < C.row_ptr[t + 1] && C.col[q] < t; ++q) {
        pp.push_back({q, C.col[q]});
        l = std::max(l, lv[C.col[q]]);
      }
      if (pp.empty()) continue;
      lv[t] = l + 1;
      tk.push_back({l + 1, T});
      prs.push_back(pp);
    }
    std::vector<int> idx(tk.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return tk[a].first < tk[b].first; });
    int L = tk.empty() ? 0 : tk[idx.back()].first;
    C.fwd_level_ptr.assign(L + 1, 0);
    for (int a : idx) {
      Task T = tk[a].second;
      T.pbeg = (int)C.fwd_pa.size();
      for (auto& pr : prs[a]) {
        C.fwd_pa.push_back(pr.first);
        C.fwd_pb.push_back(pr.second);
      }
      T.pend = (int)C.fwd_pa.size();
      C.fwd_tasks.push_back(T);
      C.fwd_level_ptr[tk[a].first]++;
    }
    for (int l = 1; l <= L; ++l) C.fwd_level_ptr[l] += C.fwd_level_ptr[l - 1];
  }
  {
    // backward: x_t = (x_t - sum_{j > t} u_tj x_j) / u_tt
    std::vector<int> lv(N, 0);
    std::vector<std::pair<int, Task>> tk;
    std::vector<std::vector<std::pair<int, int>>> prs;
    for (int t = N - 1; t >= 0; --t) {
      Task T{t, C.diag[t], 0, 0};
      std::vector<std::pair<int, int>> pp;
      int l = 0;
      for (int q = C.row_ptr[t]; q < C.row_ptr[t + 1]; ++q)
        if (C.col[q] > t) {
          pp.push_back({q, C.col[q]});
          l = std::max(l, lv[C.col[q]]);
        }
      lv[t] = l + 1;
      tk.push_back({l + 1, T});
      prs.push_back(pp);
    }
    std::vector<int> idx(tk.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return tk[a].first < tk[b].first; });
    int L = tk.empty() ? 0 : tk[idx.back()].first;
    C.bwd_level_ptr.assign(L + 1, 0);
    for (int a : idx) {
      Task T = tk[a].second;
      T.pbeg = (int)C.bwd_pa.size();
      for (auto& pr : prs[a]) {
        C.bwd_pa.push_back(pr.first);
        C.bwd_pb.push_back(pr.second);
      }
      T.pend = (int)C.bwd_pa.size();
      C.bwd_tasks.push_back(T);
      C.bwd_level_ptr[tk[a].first]++;
    }
    for (int l = 1; l <= L; ++l) C.bwd_level_ptr[l] += C.bwd_level_ptr[l - 1];
  }
  return "";
}

// Reorders (dst, payload) items so that consecutive items go to different destinations
// where possible: the first item of every destination, then the second, and so on. Items
// of one level run one per lane, and lanes of one instruction that accumulate into the
// same entry are serialized by the LDS.
template <class T>
static std::vector<std::pair<int, T>> interleave_by_dst(const std::vector<std::pair<int, T>>& in) {
  std::vector<int> order;
  std::vector<std::vector<T>> groups;
  std::vector<int> where;
  for (auto& e : in) {
    if ((int)where.size() <= e.first) where.resize(e.first + 1, -1);
    if (where[e.first] < 0) {
      where[e.first] = (int)groups.size();
      groups.emplace_back();
      order.push_back(e.first);
    }
    groups[where[e.first]].push_back(e.second);
  }
  std::vector<std::pair<int, T>> out;
  out.reserve(in.size());
  for (size_t k = 0; out.size() < in.size(); ++k)
    for (size_t g = 0; g < groups.size(); ++g)
      if (k < groups[g].size()) out.push_back({order[g], groups[g][k]});
  return out;
}

// Splits one level's (dst, payload) terms into `lists` per-wavefront lists: all terms of a
// destination go to one list (largest destinations first, to the least-loaded list), each
// list interleaved by destination. With one list per wavefront of the cell's group, a
// destination's terms accumulate in one wavefront in a fixed order.
template <class T>
static std::vector<std::vector<std::pair<int, T>>> split_by_wave(
    const std::vector<std::pair<int, T>>& in, int lists) {
  std::vector<std::vector<std::pair<int, T>>> out(lists);
  if (lists == 1) {
    out[0] = interleave_by_dst(in);
    return out;
  }
  std::vector<int> order;
  std::vector<std::vector<T>> groups;
  std::vector<int> where;
  for (auto& e : in) {
    if ((int)where.size() <= e.first) where.resize(e.first + 1, -1);
    if (where[e.first] < 0) {
      where[e.first] = (int)groups.size();
      groups.emplace_back();
      order.push_back(e.first);
    }
    groups[where[e.first]].push_back(e.second);
  }
  std::vector<int> idx(groups.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return groups[a].size() > groups[b].size(); });
  std::vector<size_t> load(lists, 0);
  for (int g : idx) {
    const int a = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    for (auto& v : groups[g]) out[a].push_back({order[g], v});
    load[a] += groups[g].size();
  }
  for (auto& l : out) l = interleave_by_dst(l);
  return out;
}

StageBlock build_stage_block(const Compiled& C, int wave_lists, bool use_tail) {
  StageBlock sb;
  const int N = C.n_state, Z = C.nnz, R = C.n_rxn;
  if (N >= 1023 || Z > 65535 || (wave_lists != 1 && wave_lists != 2 && wave_lists != 4)) return sb;
  sb.wave_lists = wave_lists;
  // dense tail of this layout: the last K positions (K <= the pattern's dense block)
  const int K = use_tail ? std::min(C.tail_k, max_tail(wave_lists)) : 0;
  const int ts = N - K;
  sb.tail_k = K;
  sb.tail_s = ts;
  std::vector<int> row_of(Z);
  for (int i = 0; i < N; ++i)
    for (int q = C.row_ptr[i]; q < C.row_ptr[i + 1]; ++q) row_of[q] = i;
  auto in_tail = [&](int q) { return row_of[q] >= ts && C.col[q] >= ts; };
  std::vector<uint8_t>& b = sb.bytes;
  auto put = [&](const void* src, size_t n) {
    size_t off = (b.size() + 15) / 16 * 16;
    b.resize(off + n);
    if (n) std::memcpy(b.data() + off, src, n);
    return (int)off;
  };
  // reactants packed 3 x 10 bits, 0x3FF = none
  std::vector<uint32_t> rx(R);
  for (int k = 0; k < R; ++k) {
    uint32_t v = 0;
    for (int o = 0; o < 3; ++o) {
      int s = C.rx_react[3 * k + o];
      v |= (uint32_t)(s < 0 ? 0x3FF : s) << (10 * o);
    }
    rx[k] = v;
  }
  sb.off_rx = put(rx.data(), 4 * rx.size());
  std::vector<uint16_t> dg(C.diag.begin(), C.diag.end());
  sb.off_diag = put(dg.data(), 2 * dg.size());
  // triangular solves: the product terms of each level (levels without terms dropped). With
  // a dense tail, tail rows keep only their terms from head columns in the forward sweep
  // and none in the backward sweep; levels are recomputed from the remaining dependences
  // (the tasks are stored in a topological order, and without a tail nothing changes).
  auto solve_terms = [&](const std::vector<Task>& tasks, const std::vector<int>& pa,
                         const std::vector<int>& pb, bool forward, int& off, int& off_lp,
                         int& n_lev) {
    std::vector<int> lv(N, 0);
    std::vector<std::pair<int, std::vector<int>>> kept;   // (level, pair indices) per task
    std::vector<int> kdst;
    for (const Task& x : tasks) {
      if (!forward && x.dst >= ts) continue;
      std::vector<int> qs;
      int l = 0;
      for (int q = x.pbeg; q < x.pend; ++q) {
        if (forward && x.dst >= ts && pb[q] >= ts) continue;
        qs.push_back(q);
        l = std::max(l, lv[pb[q]]);
      }
      if (forward && qs.empty()) continue;
      lv[x.dst] = l + 1;
      kept.push_back({l + 1, std::move(qs)});
      kdst.push_back(x.dst);
    }
    std::vector<int> idx(kept.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return kept[a].first < kept[c].first; });
    std::vector<uint32_t> t, lp(1, 0);
    n_lev = 0;
    for (size_t a = 0; a < idx.size();) {
      const int level = kept[idx[a]].first;
      std::vector<std::pair<int, int>> lvl;
      for (; a < idx.size() && kept[idx[a]].first == level; ++a)
        for (int q : kept[idx[a]].second) lvl.push_back({kdst[idx[a]], q});
      if (lvl.empty()) continue;
      for (auto& list : split_by_wave(lvl, wave_lists)) {
        for (auto& e : list) {
          t.push_back((uint32_t)e.first | ((uint32_t)pb[e.second] << 16));
          t.push_back((uint32_t)pa[e.second]);
        }
        lp.push_back((uint32_t)(t.size() / 2));
      }
      ++n_lev;
    }
    off = put(t.data(), 4 * t.size());
    off_lp = put(lp.data(), 4 * lp.size());
  };
  solve_terms(C.fwd_tasks, C.fwd_pa, C.fwd_pb, true, sb.off_sf, sb.off_sf_lp, sb.n_sf_lev);
  solve_terms(C.bwd_tasks, C.bwd_pa, C.bwd_pb, false, sb.off_sb, sb.off_sb_lp, sb.n_sb_lev);
  // LU: product terms and finalize entries per level. Entries of a dense tail keep only
  // their products over head pivots and get no finalize entry (they become the Schur
  // complement, inverted afterwards); levels are recomputed as for the sweeps.
  std::vector<char> is_diag(Z, 0), touched(Z, 0);
  for (int t = 0; t < N; ++t) is_diag[C.diag[t]] = 1;
  struct LuTask {
    int dst, diag, level;
    std::vector<int> qs;
  };
  std::vector<LuTask> lu;
  {
    std::vector<int> lev(Z, 0);
    for (const Task& x : C.lu_tasks) {
      const bool tail = in_tail(x.dst);
      LuTask u{x.dst, tail ? -1 : x.diag, 0, {}};
      int l = 0;
      for (int q = x.pbeg; q < x.pend; ++q) {
        if (tail && C.col[C.lu_pa[q]] >= ts) continue;
        u.qs.push_back(q);
        l = std::max(l, std::max(lev[C.lu_pa[q]], lev[C.lu_pb[q]]));
      }
      if (u.diag >= 0) l = std::max(l, lev[u.diag]);
      if (u.qs.empty() && u.diag < 0) continue;   // value final as assembled
      u.level = l + 1;
      lev[x.dst] = u.level;
      touched[x.dst] = 1;
      lu.push_back(std::move(u));
    }
    std::stable_sort(lu.begin(), lu.end(), [](const LuTask& a, const LuTask& c) { return a.level < c.level; });
  }
  std::vector<uint32_t> lt, ltp(1, 0), lf, lfp(1, 0);
  for (int t = 0; t < ts; ++t)
    if (!touched[C.diag[t]]) lf.push_back((uint32_t)C.diag[t] | (0xFFFFu << 16));
  lfp.push_back((uint32_t)lf.size());
  sb.n_lu_lev = lu.empty() ? 0 : lu.back().level;
  for (size_t a = 0; a < lu.size();) {
    const size_t a0 = a;
    const int level = lu[a].level;
    std::vector<std::pair<int, int>> lv;
    for (; a < lu.size() && lu[a].level == level; ++a)
      for (int q : lu[a].qs) lv.push_back({lu[a].dst, q});
    for (auto& list : split_by_wave(lv, wave_lists)) {
      for (auto& e : list) {
        lt.push_back((uint32_t)e.first | ((uint32_t)C.lu_pa[e.second] << 16));
        lt.push_back((uint32_t)C.lu_pb[e.second]);
      }
      ltp.push_back((uint32_t)(lt.size() / 2));
    }
    for (size_t i = a0; i < a; ++i) {
      const LuTask& x = lu[i];
      if (x.diag >= 0)
        lf.push_back((uint32_t)x.dst | ((uint32_t)x.diag << 16));
      else if (is_diag[x.dst] && row_of[x.dst] < ts)
        lf.push_back((uint32_t)x.dst | (0xFFFFu << 16));
    }
    lfp.push_back((uint32_t)lf.size());
  }
  if (lu.empty()) sb.n_lu_lev = 0;
  sb.off_lt = put(lt.data(), 4 * lt.size());
  sb.off_lt_lp = put(ltp.data(), 4 * ltp.size());
  sb.off_lf = put(lf.data(), 4 * lf.size());
  sb.off_lf_lp = put(lfp.data(), 4 * lfp.size());
  // row scaling of the strict upper factor
  std::vector<uint32_t> us;
  for (int t = 0; t < ts; ++t)
    for (int q = C.diag[t] + 1; q < C.row_ptr[t + 1]; ++q)
      us.push_back((uint32_t)q | ((uint32_t)C.diag[t] << 16));
  sb.n_us = (int)us.size();
  sb.off_us = put(us.data(), 4 * us.size());
  // dense tail: the terms of t = S^-1 x[s..N), whole rows per wavefront list
  {
    std::vector<std::pair<int, uint32_t>> tt;
    for (int i = 0; i < K; ++i) {
      const int r = ts + i;
      const int q0 = C.row_ptr[r + 1] - K;   // the row's last K entries are its tail columns
      if (q0 < C.row_ptr[r] || C.col[q0] != ts) return StageBlock{};
      for (int j = 0; j < K; ++j) tt.push_back({i, (uint32_t)(q0 + j) | ((uint32_t)i << 16) | ((uint32_t)j << 24)});
    }
    std::vector<uint32_t> te, tp(1, 0);
    for (auto& list : split_by_wave(tt, wave_lists)) {
      if ((int)list.size() > kWaveLanes * kTailPerLane) return StageBlock{};
      for (auto& e : list) te.push_back(e.second);
      tp.push_back((uint32_t)te.size());
    }
    sb.n_tail = (int)te.size();
    sb.off_tail = put(te.data(), 4 * te.size());
    sb.off_tail_lp = put(tp.data(), 4 * tp.size());
    std::vector<uint16_t> rs(K);
    for (int i = 0; i < K; ++i) rs[i] = (uint16_t)(C.row_ptr[ts + i + 1] - K);
    sb.off_tail_rs = put(rs.data(), 2 * rs.size());
  }
  b.resize((b.size() + 15) / 16 * 16);
  sb.core_bytes = (int)b.size();
  // extension: forcing terms and Jacobian contributions as flat term lists
  if (C.n_partials >= 65536 || R >= 65536) return StageBlock{};
  std::vector<std::pair<int, int>> ft, jt;
  for (int t = 0; t < N; ++t)
    for (int q = C.term_ptr[t]; q < C.term_ptr[t + 1]; ++q) ft.push_back({t, q});
  for (int z = 0; z < Z; ++z)
    for (int q = C.jc_ptr[z]; q < C.jc_ptr[z + 1]; ++q) jt.push_back({z, q});
  std::vector<uint32_t> fi, ji, fp(1, 0), jp(1, 0);
  std::vector<double> fc, jcf;
  for (auto& list : split_by_wave(ft, wave_lists)) {
    for (auto& e : list) {
      fi.push_back((uint32_t)e.first | ((uint32_t)C.term_rxn[e.second] << 16));
      fc.push_back(C.term_coef[e.second]);
    }
    fp.push_back((uint32_t)fi.size());
  }
  for (auto& list : split_by_wave(jt, wave_lists)) {
    for (auto& e : list) {
      ji.push_back((uint32_t)e.first | ((uint32_t)C.jc_part[e.second] << 16));
      jcf.push_back(C.jc_coef[e.second]);
    }
    jp.push_back((uint32_t)ji.size());
  }
  sb.n_ft = (int)fi.size();
  sb.n_jt = (int)ji.size();
  sb.off_ft_coef = put(fc.data(), 8 * fc.size());
  sb.off_jt_coef = put(jcf.data(), 8 * jcf.size());
  sb.off_ft = put(fi.data(), 4 * fi.size());
  sb.off_jt = put(ji.data(), 4 * ji.size());
  sb.off_ft_lp = put(fp.data(), 4 * fp.size());
  sb.off_jt_lp = put(jp.data(), 4 * jp.size());
  b.resize((b.size() + 15) / 16 * 16);
  sb.ok = true;
  return sb;
}

}  // namespace camp

namespace camp {

bool emulate_factor_solve(const Compiled& C, const StageBlock& sb, double* M, double* x) {
  const int N = C.n_state, W = sb.wave_lists, K = sb.tail_k, ts = sb.tail_s;
  auto u32 = [&](int off, int i) {
    uint32_t v;
    std::memcpy(&v, sb.bytes.data() + off + 4 * (size_t)i, 4);
    return v;
  };
  bool ok = true;
  auto inv = [&](double& v) {
    if (!(std::fabs(v) > 0.0) || !std::isfinite(v)) ok = false;
    v = 1.0 / v;
  };
  auto finalize = [&](int lo, int hi) {
    for (int i = lo; i < hi; ++i) {
      const uint32_t e = u32(sb.off_lf, i);
      const int dst = e & 0xFFFF, pv = e >> 16;
      if (pv == 0xFFFF) inv(M[dst]);
      else M[dst] *= M[pv];
    }
  };
  // factorization levels
  finalize((int)u32(sb.off_lf_lp, 0), (int)u32(sb.off_lf_lp, 1));
  for (int l = 0; l < sb.n_lu_lev; ++l) {
    for (int i = (int)u32(sb.off_lt_lp, W * l); i < (int)u32(sb.off_lt_lp, W * l + W); ++i) {
      const uint32_t a = u32(sb.off_lt, 2 * i), c = u32(sb.off_lt, 2 * i + 1);
      M[a & 0xFFFF] -= M[a >> 16] * M[c];
    }
    finalize((int)u32(sb.off_lf_lp, l + 1), (int)u32(sb.off_lf_lp, l + 2));
  }
  for (int i = 0; i < sb.n_us; ++i) {
    const uint32_t e = u32(sb.off_us, i);
    M[e & 0xFFFF] *= M[e >> 16];
  }
  // Gauss-Jordan inversion of the tail block in place
  std::vector<int> slot((size_t)K * K);
  for (int i = 0; i < sb.n_tail; ++i) {
    const uint32_t e = u32(sb.off_tail, i);
    const int r = (e >> 16) & 0xFF, c = e >> 24;
    uint16_t rs;
    std::memcpy(&rs, sb.bytes.data() + sb.off_tail_rs + 2 * (size_t)r, 2);
    if ((int)(e & 0xFFFF) != rs + c) return false;   // row-start table disagrees
    slot[(size_t)r * K + c] = (int)(e & 0xFFFF);
  }
  for (int p = 0; p < K; ++p) {
    const double piv = M[slot[(size_t)p * K + p]];
    if (!(std::fabs(piv) > 0.0) || !std::isfinite(piv)) ok = false;
    const double r = 1.0 / piv;
    std::vector<double> row(K), col(K);
    for (int j = 0; j < K; ++j) row[j] = M[slot[(size_t)p * K + j]];
    for (int i = 0; i < K; ++i) col[i] = M[slot[(size_t)i * K + p]];
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) {
        double& a = M[slot[(size_t)i * K + j]];
        if (i == p) a = j == p ? r : row[j] * r;
        else if (j == p) a = -col[i] * r;
        else a = a - col[i] * row[j] * r;
      }
  }
  for (int t = 0; t < ts; ++t)
    if (!(std::fabs(M[C.diag[t]]) > 0.0) || !std::isfinite(M[C.diag[t]])) ok = false;
  // solve
  auto sweep = [&](int off, int off_lp, int n_lev) {
    for (int l = 0; l < n_lev; ++l)
      for (int i = (int)u32(off_lp, W * l); i < (int)u32(off_lp, W * l + W); ++i) {
        const uint32_t a = u32(off, 2 * i), c = u32(off, 2 * i + 1);
        x[a & 0xFFFF] -= M[c] * x[a >> 16];
      }
  };
  sweep(sb.off_sf, sb.off_sf_lp, sb.n_sf_lev);
  std::vector<double> t(K, 0.0);
  for (int i = 0; i < sb.n_tail; ++i) {
    const uint32_t e = u32(sb.off_tail, i);
    t[(e >> 16) & 0xFF] += M[e & 0xFFFF] * x[ts + (e >> 24)];
  }
  for (int r = 0; r < ts; ++r) x[r] *= M[C.diag[r]];
  for (int i = 0; i < K; ++i) x[ts + i] = t[i];
  sweep(sb.off_sb, sb.off_sb_lp, sb.n_sb_lev);
  (void)N;
  return ok;
}

}  // namespace camp

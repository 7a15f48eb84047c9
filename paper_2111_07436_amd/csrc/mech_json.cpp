// JSON mechanism description (paper Sect. 2.3: a mechanism is described at run time in JSON,
// so species, phases and processes change without recompiling). A small JSON reader and the
// mapping of one document onto the camp_species / camp_phase / camp_reaction arrays that
// camp_mech_load takes.
//
// Document layout (keys with units are literal):
// {
//   "species":   [ {"name": "O3", "phase": "gas", "molecular weight [kg mol-1]": 0.048,
//                   "diffusion coeff [m2 s-1]": 1.5e-5, "accommodation coefficient": 0.1},
//                  {"name": "P1_org", "phase": "organic"}, ... ],
//   "phases":    [ {"name": "organic", "species": ["P1_org", ...], "density [kg m-3]": 1400,
//                   "absorber molecular weight [kg mol-1]": 0.2,
//                   "radius from state": false}, ... ],
//   "aerosol representation": {"type": "sections", "instances": {"organic": 8, ...}},
//   "processes": [ {"type": "ARRHENIUS", "reactants": {"O3": 1, "NO": 1},
//                   "products": {"NO2": 1.0}, "A": 3e-12, "Ea/kb [K]": 1500}, ... ]
// }
// Species in a phase are listed by that phase; "phase": "gas" (or no phase) is gas phase.
// Reactant values are integer multiplicities, product values molar yields. Process keys by
// type (missing optional keys default to 0 unless stated):
//   ARRHENIUS, CONDENSED_PHASE_ARRHENIUS: "A", "Ea/kb [K]", "B", "D [K]" (300), "E [Pa-1]";
//       condensed: "phase", "aqueous" (false)
//   PHOTOLYSIS: "J0 [s-1]", "scale by cos(sza)" (false); EMISSION: "rate [mol m-3 s-1]";
//   FIRST_ORDER_LOSS: "rate constant [s-1]"
//   HENRYS_LAW_PHASE_TRANSFER: "phase", "gas species", "aerosol species", "H298 [M Pa-1]", "C [K]"
//   SIMPOL_PHASE_TRANSFER: "phase", "gas species", "aerosol species", "B" ([B1, B2, B3, B4]),
//     "full Raoult" (false: the fixed absorber amount only)
//   TROE: "k0" and "kinf" ({"A", "Ea/kb [K]", "B"}), "Fc" (0.6), "N" (1.0)
//   CUSTOM_H2O2: "k1", "k2"; CUSTOM_OH_HNO3: "k0", "k2", "k3" (each {"A", "Ea/kb [K]", "B"})
//   WENNBERG_TUNNELING: "A", "B [K]", "C [K3]"
//   AQUEOUS_REVERSIBLE: "phase", "A", "C [K]", "k_reverse"
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "mech.hpp"

namespace camp {
namespace {

struct JVal {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  bool b = false;
  double num = 0.0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;   // in document order

  const JVal* get(const std::string& k) const {
    for (auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct Parser {
  const char* p;
  const char* end;
  std::string err;

  void ws() {
    while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
  }
  bool fail(const std::string& m) {
    if (err.empty()) err = m;
    return false;
  }
  bool lit(const char* s) {
    const size_t n = std::strlen(s);
    if ((size_t)(end - p) < n || std::strncmp(p, s, n) != 0) return false;
    p += n;
    return true;
  }
  bool string(std::string& out) {
    if (p >= end || *p != '"') return fail("expected a string");
    ++p;
    out.clear();
    while (p < end && *p != '"') {
      char c = *p++;
      if (c == '\\') {
        if (p >= end) return fail("unterminated escape");
        const char e = *p++;
        switch (e) {
          case '"': out += '"'; break;
          case '\\': out += '\\'; break;
          case '/': out += '/'; break;
          case 'b': out += '\b'; break;
          case 'f': out += '\f'; break;
          case 'n': out += '\n'; break;
          case 'r': out += '\r'; break;
          case 't': out += '\t'; break;
          case 'u': {
            if (end - p < 4) return fail("bad \\u escape");
            const unsigned v = (unsigned)std::strtoul(std::string(p, 4).c_str(), nullptr, 16);
            p += 4;
            if (v < 0x80) {
              out += (char)v;
            } else if (v < 0x800) {
              out += (char)(0xC0 | (v >> 6));
              out += (char)(0x80 | (v & 0x3F));
            } else {
              out += (char)(0xE0 | (v >> 12));
              out += (char)(0x80 | ((v >> 6) & 0x3F));
              out += (char)(0x80 | (v & 0x3F));
            }
            break;
          }
          default: return fail("bad escape");
        }
      } else {
        out += c;
      }
    }
    if (p >= end) return fail("unterminated string");
    ++p;
    return true;
  }
  bool value(JVal& v, int depth) {
    if (depth > 64) return fail("nesting too deep");
    ws();
    if (p >= end) return fail("unexpected end of document");
    const char c = *p;
    if (c == '{') {
      ++p;
      v.kind = JVal::OBJ;
      ws();
      if (p < end && *p == '}') { ++p; return true; }
      while (true) {
        ws();
        std::string k;
        if (!string(k)) return false;
        ws();
        if (p >= end || *p != ':') return fail("expected ':'");
        ++p;
        JVal x;
        if (!value(x, depth + 1)) return false;
        v.obj.emplace_back(std::move(k), std::move(x));
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == '}') { ++p; return true; }
        return fail("expected ',' or '}'");
      }
    }
    if (c == '[') {
      ++p;
      v.kind = JVal::ARR;
      ws();
      if (p < end && *p == ']') { ++p; return true; }
      while (true) {
        JVal x;
        if (!value(x, depth + 1)) return false;
        v.arr.push_back(std::move(x));
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == ']') { ++p; return true; }
        return fail("expected ',' or ']'");
      }
    }
    if (c == '"') {
      v.kind = JVal::STR;
      return string(v.str);
    }
    if (lit("true")) { v.kind = JVal::BOOL; v.b = true; return true; }
    if (lit("false")) { v.kind = JVal::BOOL; v.b = false; return true; }
    if (lit("null")) { v.kind = JVal::NUL; return true; }
    char* q = nullptr;
    const std::string tail(p, std::min<size_t>(end - p, 64));
    const double d = std::strtod(tail.c_str(), &q);
    if (q == tail.c_str()) return fail("unexpected character");
    p += q - tail.c_str();
    v.kind = JVal::NUM;
    v.num = d;
    return true;
  }
};

// Reads a number (default `def` when absent); false if present and not a number.
bool number(const JVal& o, const char* key, double def, double* out) {
  const JVal* v = o.get(key);
  if (!v) { *out = def; return true; }
  if (v->kind == JVal::NUM) { *out = v->num; return true; }
  if (v->kind == JVal::BOOL) { *out = v->b ? 1.0 : 0.0; return true; }
  return false;
}

}  // namespace

std::string parse_mechanism_json(const char* text, size_t len, MechDescription& out) {
  Parser ps{text, text + len, ""};
  JVal doc;
  if (!ps.value(doc, 0)) {
    std::ostringstream e;
    e << "JSON: " << ps.err << " at offset " << (ps.p - text);
    return e.str();
  }
  ps.ws();
  if (ps.p != ps.end) return "JSON: trailing characters after the document";
  if (doc.kind != JVal::OBJ) return "JSON: the document must be an object";
  const JVal* sp = doc.get("species");
  const JVal* ph = doc.get("phases");
  const JVal* pr = doc.get("processes");
  if (!sp || sp->kind != JVal::ARR || sp->arr.empty()) return "JSON: \"species\" must be a non-empty array";
  if (ph && ph->kind != JVal::ARR) return "JSON: \"phases\" must be an array";
  if (!pr || pr->kind != JVal::ARR) return "JSON: \"processes\" must be an array";

  std::map<std::string, int> sid, pid;
  out = MechDescription{};
  std::vector<std::string> sphase;
  for (const JVal& s : sp->arr) {
    const JVal* nm = s.get("name");
    if (s.kind != JVal::OBJ || !nm || nm->kind != JVal::STR) return "JSON: every species needs a \"name\"";
    if (sid.count(nm->str)) return "JSON: duplicate species \"" + nm->str + "\"";
    sid[nm->str] = (int)out.species.size();
    MechDescription::Species x;
    x.name = nm->str;
    const JVal* p = s.get("phase");
    sphase.push_back(p && p->kind == JVal::STR ? p->str : "gas");
    if (!number(s, "molecular weight [kg mol-1]", 0.1, &x.mw) ||
        !number(s, "diffusion coeff [m2 s-1]", 1e-5, &x.diff) ||
        !number(s, "accommodation coefficient", 0.1, &x.accom))
      return "JSON: species \"" + nm->str + "\" has a non-numeric property";
    out.species.push_back(x);
  }
  const JVal* rep = doc.get("aerosol representation");
  const JVal* inst = rep ? rep->get("instances") : nullptr;
  if (ph) {
    for (const JVal& q : ph->arr) {
      const JVal* nm = q.get("name");
      const JVal* ls = q.get("species");
      if (q.kind != JVal::OBJ || !nm || nm->kind != JVal::STR || !ls || ls->kind != JVal::ARR)
        return "JSON: every phase needs a \"name\" and a \"species\" array";
      if (pid.count(nm->str) || nm->str == "gas") return "JSON: bad or duplicate phase \"" + nm->str + "\"";
      pid[nm->str] = (int)out.phases.size();
      MechDescription::Phase x;
      x.name = nm->str;
      for (const JVal& e : ls->arr) {
        if (e.kind != JVal::STR || !sid.count(e.str))
          return "JSON: phase \"" + nm->str + "\" lists an unknown species";
        x.species.push_back(sid[e.str]);
      }
      double n = 1.0;
      const JVal* ni = inst ? inst->get(nm->str) : nullptr;
      if (ni && ni->kind == JVal::NUM) n = ni->num;
      if (!(n >= 1.0) || n != std::floor(n)) return "JSON: phase \"" + nm->str + "\" needs a positive integer instance count";
      x.n_instances = (int)n;
      double grows = 0.0;
      if (!number(q, "density [kg m-3]", 1000.0, &x.density) ||
          !number(q, "absorber molecular weight [kg mol-1]", 0.2, &x.mw_absorber) ||
          !number(q, "radius from state", 0.0, &grows))
        return "JSON: phase \"" + nm->str + "\" has a non-numeric property";
      x.radius_from_state = grows != 0.0 ? 1 : 0;
      out.phases.push_back(x);
    }
  }
  for (size_t s = 0; s < out.species.size(); ++s) {
    if (sphase[s] == "gas") {
      out.species[s].phase = -1;
    } else if (pid.count(sphase[s])) {
      out.species[s].phase = pid[sphase[s]];
    } else {
      return "JSON: species \"" + out.species[s].name + "\" names an unknown phase \"" + sphase[s] + "\"";
    }
  }

  static const std::map<std::string, int> kTypes = {
      {"ARRHENIUS", CAMP_RXN_ARRHENIUS}, {"PHOTOLYSIS", CAMP_RXN_PHOTOLYSIS},
      {"EMISSION", CAMP_RXN_EMISSION}, {"FIRST_ORDER_LOSS", CAMP_RXN_FIRST_ORDER_LOSS},
      {"CONDENSED_PHASE_ARRHENIUS", CAMP_RXN_CONDENSED_ARRHENIUS},
      {"HENRYS_LAW_PHASE_TRANSFER", CAMP_RXN_HENRY_TRANSFER},
      {"SIMPOL_PHASE_TRANSFER", CAMP_RXN_SIMPOL_TRANSFER}, {"TROE", CAMP_RXN_TROE},
      {"CUSTOM_H2O2", CAMP_RXN_CUSTOM_H2O2}, {"CUSTOM_OH_HNO3", CAMP_RXN_CUSTOM_OH_HNO3},
      {"WENNBERG_TUNNELING", CAMP_RXN_WENNBERG_TUNNELING},
      {"AQUEOUS_REVERSIBLE", CAMP_RXN_AQUEOUS_REVERSIBLE}};
  int idx = 0;
  for (const JVal& q : pr->arr) {
    std::ostringstream where;
    where << "JSON: process " << idx++;
    const JVal* ty = q.get("type");
    if (q.kind != JVal::OBJ || !ty || ty->kind != JVal::STR || !kTypes.count(ty->str))
      return where.str() + " needs a known \"type\"";
    camp_reaction r{};
    r.type = kTypes.at(ty->str);
    r.phase = -1;
    const JVal* phn = q.get("phase");
    if (phn) {
      if (phn->kind != JVal::STR || !pid.count(phn->str)) return where.str() + " names an unknown phase";
      r.phase = pid[phn->str];
    }
    auto species_of = [&](const JVal* v, int* id) {
      if (!v || v->kind != JVal::STR || !sid.count(v->str)) return false;
      *id = sid[v->str];
      return true;
    };
    if (r.type == CAMP_RXN_HENRY_TRANSFER || r.type == CAMP_RXN_SIMPOL_TRANSFER) {
      if (!species_of(q.get("gas species"), &r.react[0]) || !species_of(q.get("aerosol species"), &r.prod[0]))
        return where.str() + " needs \"gas species\" and \"aerosol species\"";
      r.n_react = r.n_prod = 1;
      r.yield[0] = 1.0;
    } else {
      const JVal* re = q.get("reactants");
      const JVal* pd = q.get("products");
      if ((re && re->kind != JVal::OBJ) || (pd && pd->kind != JVal::OBJ))
        return where.str() + ": \"reactants\" and \"products\" must be objects";
      if (re)
        for (auto& kv : re->obj) {
          if (!sid.count(kv.first)) return where.str() + " has an unknown reactant \"" + kv.first + "\"";
          double n = 1.0;
          if (kv.second.kind == JVal::NUM) n = kv.second.num;
          else if (kv.second.kind == JVal::OBJ && !number(kv.second, "qty", 1.0, &n))
            return where.str() + ": bad reactant quantity";
          if (!(n >= 1.0) || n != std::floor(n)) return where.str() + ": reactant quantities are positive integers";
          for (int c = 0; c < (int)n; ++c) {
            if (r.n_react >= 3) return where.str() + ": at most 3 reactant occurrences";
            r.react[r.n_react++] = sid[kv.first];
          }
        }
      if (pd)
        for (auto& kv : pd->obj) {
          if (!sid.count(kv.first)) return where.str() + " has an unknown product \"" + kv.first + "\"";
          double y = 1.0;
          if (kv.second.kind == JVal::NUM) y = kv.second.num;
          else if (kv.second.kind == JVal::OBJ && !number(kv.second, "yield", 1.0, &y))
            return where.str() + ": bad product yield";
          if (r.n_prod >= 3) return where.str() + ": at most 3 products";
          r.prod[r.n_prod] = sid[kv.first];
          r.yield[r.n_prod++] = y;
        }
    }
    auto arr3 = [&](const char* key, double* dst) {
      const JVal* o = q.get(key);
      if (!o || o->kind != JVal::OBJ) return false;
      return number(*o, "A", 0.0, &dst[0]) && number(*o, "Ea/kb [K]", 0.0, &dst[1]) &&
             number(*o, "B", 0.0, &dst[2]);
    };
    bool ok = true;
    double* p = r.p;
    switch (r.type) {
      case CAMP_RXN_ARRHENIUS:
      case CAMP_RXN_CONDENSED_ARRHENIUS:
        ok = number(q, "A", 0.0, &p[0]) && number(q, "Ea/kb [K]", 0.0, &p[1]) &&
             number(q, "B", 0.0, &p[2]) && number(q, "D [K]", 300.0, &p[3]) &&
             number(q, "E [Pa-1]", 0.0, &p[4]) && number(q, "aqueous", 0.0, &p[5]);
        break;
      case CAMP_RXN_PHOTOLYSIS:
        ok = number(q, "J0 [s-1]", 0.0, &p[0]) && number(q, "scale by cos(sza)", 0.0, &p[1]);
        break;
      case CAMP_RXN_EMISSION: ok = number(q, "rate [mol m-3 s-1]", 0.0, &p[0]); break;
      case CAMP_RXN_FIRST_ORDER_LOSS: ok = number(q, "rate constant [s-1]", 0.0, &p[0]); break;
      case CAMP_RXN_HENRY_TRANSFER:
        ok = number(q, "H298 [M Pa-1]", 0.0, &p[0]) && number(q, "C [K]", 0.0, &p[1]);
        break;
      case CAMP_RXN_SIMPOL_TRANSFER: {
        const JVal* b = q.get("B");
        ok = b && b->kind == JVal::ARR && b->arr.size() == 4;
        for (int k = 0; ok && k < 4; ++k) {
          ok = b->arr[k].kind == JVal::NUM;
          if (ok) p[k] = b->arr[k].num;
        }
        ok = ok && number(q, "full Raoult", 0.0, &p[4]);
        break;
      }
      case CAMP_RXN_TROE:
        ok = arr3("k0", p) && arr3("kinf", p + 3) && number(q, "Fc", 0.6, &p[6]) &&
             number(q, "N", 1.0, &p[7]);
        break;
      case CAMP_RXN_CUSTOM_H2O2: ok = arr3("k1", p) && arr3("k2", p + 3); break;
      case CAMP_RXN_CUSTOM_OH_HNO3: ok = arr3("k0", p) && arr3("k2", p + 3) && arr3("k3", p + 6); break;
      case CAMP_RXN_WENNBERG_TUNNELING:
        ok = number(q, "A", 0.0, &p[0]) && number(q, "B [K]", 0.0, &p[1]) && number(q, "C [K3]", 0.0, &p[2]);
        break;
      case CAMP_RXN_AQUEOUS_REVERSIBLE:
        ok = number(q, "A", 0.0, &p[0]) && number(q, "C [K]", 0.0, &p[1]) &&
             number(q, "k_reverse", 0.0, &p[2]);
        break;
      default: break;
    }
    if (!ok) return where.str() + " (" + ty->str + ") has missing or non-numeric parameters";
    out.reactions.push_back(r);
  }
  return "";
}

}  // namespace camp

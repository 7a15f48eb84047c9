// Host-side driver for the sanitizer test (built with g++ -fsanitize=address,undefined by
// tests/test_host_sanitize.py, no HIP): runs the mechanism front ends on every JSON document
// named on the command line, valid or damaged, and for each one that compiles, every table
// layout, the table program's host emulation, packing, unpacking, and unpacking of damaged
// packed buffers (payload bytes changed with the checksum recomputed, so the structural
// checks behind the checksum are reached). Any memory or undefined-behaviour error aborts
// the process through the sanitizer; otherwise it prints one line per document and exits 0.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "mech.hpp"

using namespace camp;

namespace {

uint64_t fnv1a(const uint8_t* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

// xorshift64: deterministic damage positions and values
uint64_t next(uint64_t& s) {
  s ^= s << 13;
  s ^= s >> 7;
  s ^= s << 17;
  return s;
}

constexpr size_t kHeader = 8 + 4 + 8 + 8;   // magic, version, payload length, checksum

int run_packed(const std::vector<uint8_t>& packed, uint64_t seed) {
  int accepted = 0;
  Compiled C;
  StageBlock st[4];
  if (!unpack_compiled(packed.data(), packed.size(), C, st).empty()) {
    std::fprintf(stderr, "an undamaged packed mechanism was rejected\n");
    return -1;
  }
  uint64_t s = seed | 1;
  for (int trial = 0; trial < 64 && packed.size() > kHeader; ++trial) {
    std::vector<uint8_t> b = packed;
    const int flips = 1 + (int)(next(s) % 4);
    for (int f = 0; f < flips; ++f) {
      const size_t at = kHeader + next(s) % (b.size() - kHeader);
      b[at] = (uint8_t)next(s);
    }
    const uint64_t sum = fnv1a(b.data() + kHeader, b.size() - kHeader);
    std::memcpy(b.data() + 20, &sum, 8);
    Compiled D;
    StageBlock sd[4];
    if (unpack_compiled(b.data(), b.size(), D, sd).empty()) ++accepted;
    // truncated buffers must be rejected
    const size_t cut = next(s) % b.size();
    Compiled E;
    StageBlock se[4];
    if (unpack_compiled(b.data(), cut, E, se).empty()) {
      std::fprintf(stderr, "a truncated packed mechanism was accepted\n");
      return -1;
    }
  }
  return accepted;
}

int run_document(const std::string& text, uint64_t seed) {
  MechDescription d;
  const std::string err = parse_mechanism_json(text.data(), text.size(), d);
  if (!err.empty()) {
    std::printf("parse error: %s\n", err.c_str());
    return 0;
  }
  std::vector<camp_species> sp(d.species.size());
  for (size_t i = 0; i < sp.size(); ++i)
    sp[i] = camp_species{d.species[i].name.c_str(), d.species[i].phase, d.species[i].mw,
                         d.species[i].diff, d.species[i].accom};
  std::vector<camp_phase> ph(d.phases.size());
  for (size_t i = 0; i < ph.size(); ++i)
    ph[i] = camp_phase{d.phases[i].name.c_str(), (int)d.phases[i].species.size(),
                       d.phases[i].species.data(), d.phases[i].n_instances, d.phases[i].density,
                       d.phases[i].mw_absorber, d.phases[i].radius_from_state};
  Compiled C;
  const std::string cerr = compile_mechanism(d.reactions.data(), (int)d.reactions.size(), sp.data(),
                                             (int)sp.size(), ph.data(), (int)ph.size(), C);
  if (!cerr.empty()) {
    std::printf("compile error: %s\n", cerr.c_str());
    return 0;
  }
  StageBlock st[4] = {build_stage_block(C, 1, true), build_stage_block(C, 2, true),
                      build_stage_block(C, 4, true), build_stage_block(C, 1, false)};
  uint64_t s = seed | 1;
  for (const StageBlock& b : st) {
    if (!b.ok) continue;
    // a diagonally dominant matrix on the filled pattern, and a right-hand side
    std::vector<double> m(C.nnz), x(C.n_state);
    for (int i = 0; i < C.n_state; ++i) {
      for (int q = C.row_ptr[i]; q < C.row_ptr[i + 1]; ++q)
        m[q] = C.col[q] == i ? 4.0 + C.row_ptr[i + 1] - C.row_ptr[i] : -(double)(next(s) % 1000) / 1000.0;
      x[i] = (double)(next(s) % 1000) / 1000.0;
    }
    if (!emulate_factor_solve(C, b, m.data(), x.data())) {
      std::fprintf(stderr, "table program failed on a diagonally dominant matrix\n");
      return -1;
    }
  }
  const std::vector<uint8_t> packed = pack_compiled(C, st);
  const int acc = run_packed(packed, seed);
  if (acc < 0) return -1;
  std::printf("ok: %d state variables, %d reactions, %zu packed bytes, %d of 64 damaged buffers "
              "passed the structural checks\n", C.n_state, C.n_rxn, packed.size(), acc);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  for (int a = 1; a < argc; ++a) {
    std::ifstream f(argv[a], std::ios::binary);
    std::stringstream ss;
    ss << f.rdbuf();
    std::printf("%s: ", argv[a]);
    if (run_document(ss.str(), 0x9E3779B97F4A7C15ull ^ (uint64_t)a) != 0) return 1;
  }
  return 0;
}

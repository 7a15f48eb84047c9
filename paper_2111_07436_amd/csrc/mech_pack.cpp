// Serialization of a compiled mechanism: one self-describing byte buffer holding every
// table the engines read, so a mechanism compiled once can be handed to other processes or
// ranks and loaded there without repeating the host compile (the paper's CampCore objects
// are packed on one process and unpacked on others, Sect. 2.1 and Sect. 2.4.2).
//
// Layout: magic "CAMPMECH", format version, byte count of the payload, FNV-1a checksum of the
// payload, then the payload: the scalar sizes, every vector as (count u64, elements), the
// four table blocks. Little-endian, as the host that wrote it (checked by the magic).
#include <cstring>
#include <string>
#include <vector>

#include "mech.hpp"

namespace camp {
namespace {

constexpr char kMagic[8] = {'C', 'A', 'M', 'P', 'M', 'E', 'C', 'H'};
constexpr uint32_t kVersion = 4;

uint64_t fnv1a(const uint8_t* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

struct Writer {
  std::vector<uint8_t> b;
  void raw(const void* p, size_t n) {
    const uint8_t* c = static_cast<const uint8_t*>(p);
    b.insert(b.end(), c, c + n);
  }
  template <class T>
  void pod(const T& v) { raw(&v, sizeof(T)); }
  template <class T>
  void vec(const std::vector<T>& v) {
    pod<uint64_t>(v.size());
    if (!v.empty()) raw(v.data(), sizeof(T) * v.size());
  }
};

struct Reader {
  const uint8_t* p;
  const uint8_t* end;
  bool ok = true;
  void raw(void* dst, size_t n) {
    if (!ok || (size_t)(end - p) < n) { ok = false; return; }
    std::memcpy(dst, p, n);
    p += n;
  }
  template <class T>
  void pod(T& v) { raw(&v, sizeof(T)); }
  template <class T>
  void vec(std::vector<T>& v) {
    uint64_t n = 0;
    pod(n);
    if (!ok || n > (uint64_t)(end - p) / sizeof(T)) { ok = false; return; }
    v.resize(n);
    if (n) raw(v.data(), sizeof(T) * n);
  }
};

template <class IO, class C, class S>
void fields(IO& io, C& c, S* stage) {
  io.pod(c.n_state); io.pod(c.n_gas); io.pod(c.n_inst); io.pod(c.n_rxn); io.pod(c.n_ext);
  io.pod(c.nnz0); io.pod(c.nnz); io.pod(c.lu_pairs); io.pod(c.tail_k); io.pod(c.nnz_lu);
  io.pod(c.n_partials);
  io.vec(c.inst_phase); io.vec(c.inst_base); io.vec(c.perm); io.vec(c.iperm);
  io.vec(c.rate); io.vec(c.rx_react); io.vec(c.rx_nr); io.vec(c.rx_pofs);
  io.vec(c.param_ptr); io.vec(c.param); io.vec(c.param_w);
  io.vec(c.term_ptr); io.vec(c.term_rxn); io.vec(c.term_coef);
  io.vec(c.row_ptr); io.vec(c.col); io.vec(c.diag); io.vec(c.pattern0);
  io.vec(c.jc_ptr); io.vec(c.jc_part); io.vec(c.jc_coef);
  io.vec(c.lu_tasks); io.vec(c.fwd_tasks); io.vec(c.bwd_tasks);
  io.vec(c.lu_level_ptr); io.vec(c.fwd_level_ptr); io.vec(c.bwd_level_ptr);
  io.vec(c.lu_pa); io.vec(c.lu_pb); io.vec(c.fwd_pa); io.vec(c.fwd_pb); io.vec(c.bwd_pa);
  io.vec(c.bwd_pb);
  for (int v = 0; v < 4; ++v) {
    auto& s = stage[v];
    io.vec(s.bytes);
    io.pod(s.core_bytes); io.pod(s.off_rx); io.pod(s.off_diag); io.pod(s.off_sf);
    io.pod(s.off_sf_lp); io.pod(s.off_sb); io.pod(s.off_sb_lp); io.pod(s.off_lt);
    io.pod(s.off_lt_lp); io.pod(s.off_lf); io.pod(s.off_lf_lp); io.pod(s.off_us);
    io.pod(s.n_sf_lev); io.pod(s.n_sb_lev); io.pod(s.n_us); io.pod(s.off_ft);
    io.pod(s.off_ft_coef); io.pod(s.off_jt); io.pod(s.off_jt_coef); io.pod(s.n_ft);
    io.pod(s.n_jt); io.pod(s.off_ft_lp); io.pod(s.off_jt_lp); io.pod(s.wave_lists);
    io.pod(s.n_lu_lev); io.pod(s.tail_k); io.pod(s.tail_s); io.pod(s.off_tail);
    io.pod(s.off_tail_lp); io.pod(s.n_tail); io.pod(s.off_tail_rs); io.pod(s.ok);
  }
}

}  // namespace

std::vector<uint8_t> pack_compiled(const Compiled& C, const StageBlock* stage) {
  Writer body;
  fields(body, C, stage);
  Writer out;
  out.raw(kMagic, sizeof(kMagic));
  out.pod(kVersion);
  out.pod<uint64_t>(body.b.size());
  out.pod<uint64_t>(fnv1a(body.b.data(), body.b.size()));
  out.raw(body.b.data(), body.b.size());
  return out.b;
}

std::string unpack_compiled(const uint8_t* buf, size_t size, Compiled& C, StageBlock* stage) {
  Reader hdr{buf, buf + size};
  char magic[8];
  uint32_t version = 0;
  uint64_t n = 0, sum = 0;
  hdr.raw(magic, sizeof(magic));
  hdr.pod(version);
  hdr.pod(n);
  hdr.pod(sum);
  if (!hdr.ok || std::memcmp(magic, kMagic, sizeof(kMagic)) != 0) return "not a packed mechanism";
  if (version != kVersion) return "packed mechanism of another format version";
  if (n != (uint64_t)(hdr.end - hdr.p)) return "packed mechanism has the wrong length";
  if (fnv1a(hdr.p, n) != sum) return "packed mechanism is corrupted (checksum)";
  Reader r{hdr.p, hdr.end};
  fields(r, C, stage);
  if (!r.ok || r.p != r.end) return "packed mechanism is truncated or malformed";
  // structural consistency of what the engines index with
  if (C.n_state < 1 || (int)C.perm.size() != C.n_state || (int)C.row_ptr.size() != C.n_state + 1 ||
      (int)C.col.size() != C.nnz || (int)C.diag.size() != C.n_state || (int)C.rate.size() != C.n_rxn ||
      (int)C.rx_react.size() != 3 * C.n_rxn || (int)C.rx_pofs.size() != C.n_rxn + 1)
    return "packed mechanism is inconsistent";
  if (C.param_ptr.empty() || C.param_ptr[0] != 0 || C.param_ptr.back() != (int)C.param.size() ||
      C.param_w.size() != C.param.size())
    return "packed mechanism is inconsistent";
  for (size_t q = 0; q + 1 < C.param_ptr.size(); ++q) {
    const int b = C.param_ptr[q], e = C.param_ptr[q + 1];
    if (e < b + kParamHead || b < 0) return "packed mechanism is inconsistent";
    const int k = C.param[b], fl = C.param[b + 1];
    if (k < 0 || k >= C.n_rxn || fl < 1 || fl > 3) return "packed mechanism is inconsistent";
    for (int i = 2; i < kParamHead; ++i) {
      const int d = C.param[b + i];
      const bool used = (i == 2) ? (fl & kParamRaoult) : (fl & kParamRadius);
      if (used && (d < 0 || d >= C.n_rxn)) return "packed mechanism is inconsistent";
    }
    if (C.rx_nr[k] != 1 || C.rx_pofs[k + 1] - C.rx_pofs[k] != 1 + n_param_partials(fl))
      return "packed mechanism is inconsistent";
    for (int i = b + kParamHead; i < e; ++i)
      if (C.param[i] < 0 || C.param[i] >= C.n_state) return "packed mechanism is inconsistent";
  }
  for (int v = 0; v < 4; ++v) {
    const StageBlock& s = stage[v];
    if (!s.ok) continue;
    const int n = (int)s.bytes.size();
    for (int off : {s.core_bytes, s.off_rx, s.off_diag, s.off_sf, s.off_sf_lp, s.off_sb, s.off_sb_lp,
                    s.off_lt, s.off_lt_lp, s.off_lf, s.off_lf_lp, s.off_us, s.off_ft, s.off_ft_coef,
                    s.off_jt, s.off_jt_coef, s.off_ft_lp, s.off_jt_lp, s.off_tail, s.off_tail_lp,
                    s.off_tail_rs})
      if (off < 0 || off > n) return "packed mechanism has a table outside its block";
  }
  return "";
}

}  // namespace camp

// Launch-shape table of the streaming kernels (host code only).
//
// One base entry, which also holds the choices fixed when buffers are laid out
// (ld_pad, op_t, k0_sym), and entries for size buckets "n <= N" that override
// only kernel shapes.  Calls on one QP (single-QP and shared-matrix entry points)
// select the bucket of that QP's n for their duration (TuneScope); batches use
// the base entry, whose shapes also size their workspaces.  The table comes from
// QPGPU_TUNE (a "key=val,..." override of the base), else from the cache written
// by paper_2104_12916_amd/autotune.py (QPGPU_AUTOTUNE_CACHE, default
// autotune_gfx950.txt beside the library; ignored on another architecture), else
// the built-in defaults.  qp_tune_set / qp_tune_get replace and print it.
#include <dlfcn.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qpgpu.h"
#include "common.hpp"

namespace qpg {
namespace {

struct TuneTable {
  Tune base;
  std::vector<std::pair<int, Tune>> buckets;  // (max n, shapes), ascending
};

thread_local const Tune* t_cur = nullptr;

// Apply "key=val,key=val" to t; alloc: whether layout keys may change.
// Returns false on an unknown key or an out-of-range value.
bool parse_keys(const std::string& spec, Tune& t, bool alloc) {
  std::stringstream ss(spec);
  std::string tok;
  while (std::getline(ss, tok, ',')) {
    if (tok.empty()) continue;
    const size_t eq = tok.find('=');
    if (eq == std::string::npos) return false;
    const std::string k = tok.substr(0, eq);
    const int v = atoi(tok.c_str() + eq + 1);
    bool ok = true;
    if (k == "rows_bpc") ok = v >= 1 && v <= kMaxRowsBpc, t.rows_bpc = v;
    else if (k == "rows_unroll") ok = v == 4 || v == 8 || v == 16, t.rows_unroll = v;
    else if (k == "cols_bpc") ok = v >= 1 && v <= kMaxColsBpc, t.cols_bpc = v;
    else if (k == "cols_unroll") ok = v == 4 || v == 8, t.cols_unroll = v;
    else if (k == "qe_stage") ok = v == 0 || v == 1, t.qe_stage = v;
    else if (k == "rows_stage") ok = v == 0 || v == 1, t.rows_stage = v;
    else if (k == "brows_stage") ok = v == 0 || v == 1, t.brows_stage = v;
    else if (k == "brows_unroll") ok = v == 4 || v == 8, t.brows_unroll = v;
    else if (k == "sym_wg") ok = v >= 1 && v <= kMaxSymWg, t.sym_wg = v;
    else if (k == "sym_units") ok = v >= 1 && v <= 64, t.sym_units = v;
    else if (k == "bsym_units") ok = v >= 1 && v <= 256, t.bsym_units = v;
    else if (k == "bsym_wave") ok = v == 0 || v == 1, t.bsym_wave = v;
    else if (k == "sym_teams") ok = v == 1 || v == 2, t.sym_teams = v;
    else if (k == "sym_rows") ok = v == 2 || v == 4, t.sym_rows = v;
    else if (k == "sym_pipe") ok = v == 0 || v == 1, t.sym_pipe = v;
    else if (k == "ld_nt") ok = v >= 0 && v <= 3, t.ld_nt = v;
    else if (k == "upd_threads") ok = v == 256 || v == 512 || v == 1024, t.upd_threads = v;
    else if (k == "mv_rt") ok = v == 1 || v == 2, t.mv_rt = v;
    else if (k == "cg_fold") ok = v >= 0 && v <= 7, t.cg_fold = v;
    else if (alloc && k == "ld_pad") ok = v >= 0 && v <= 1024 && v % 64 == 0, t.ld_pad = v;
    else if (alloc && k == "op_t") ok = v == 0 || v == 1, t.op_t = v;
    else if (alloc && k == "k0_sym") ok = v == 0 || v == 1, t.k0_sym = v;
    else ok = false;
    if (!ok) return false;
  }
  return true;
}

// Table text: "default k=v,...", "n<=N k=v,...", "arch NAME", "# comment", or a
// bare "k=v,..." line (= default).  Buckets start from the base entry.
bool parse_table(const std::string& text, TuneTable& out, std::string* arch) {
  TuneTable t;
  std::vector<std::pair<int, std::string>> bl;
  std::stringstream ss(text);
  std::string line;
  while (std::getline(ss, line)) {
    while (!line.empty() && (line.back() == '\r' || line.back() == ' ')) line.pop_back();
    size_t a = line.find_first_not_of(' ');
    if (a == std::string::npos || line[a] == '#') continue;
    line = line.substr(a);
    if (line.rfind("arch ", 0) == 0) {
      if (arch) *arch = line.substr(5);
    } else if (line.rfind("default ", 0) == 0) {
      if (!parse_keys(line.substr(8), t.base, true)) return false;
    } else if (line.rfind("n<=", 0) == 0) {
      const size_t sp = line.find(' ');
      const int nmax = atoi(line.c_str() + 3);
      if (nmax <= 0) return false;
      bl.emplace_back(nmax, sp == std::string::npos ? std::string() : line.substr(sp + 1));
    } else if (!parse_keys(line, t.base, true)) {
      return false;
    }
  }
  for (auto& b : bl) {
    Tune x = t.base;
    if (!parse_keys(b.second, x, false)) return false;
    t.buckets.emplace_back(b.first, x);
  }
  std::sort(t.buckets.begin(), t.buckets.end(), [](auto& u, auto& v) { return u.first < v.first; });
  out = t;
  return true;
}

std::string lib_dir() {
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&parse_table), &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t sl = p.rfind('/');
    if (sl != std::string::npos) return p.substr(0, sl);
  }
  return ".";
}

bool device_is(const std::string& arch) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  return std::string(prop.gcnArchName).rfind(arch, 0) == 0;
}

TuneTable& table() {
  static TuneTable t = [] {
    TuneTable v;
    if (const char* e = getenv("QPGPU_TUNE")) {
      Tune b;
      if (parse_keys(e, b, true)) v.base = b;
      return v;
    }
    const char* c = getenv("QPGPU_AUTOTUNE_CACHE");
    const std::string path = c ? std::string(c) : lib_dir() + "/autotune_gfx950.txt";
    std::ifstream f(path);
    if (!f) return v;
    std::stringstream buf;
    buf << f.rdbuf();
    TuneTable x;
    std::string arch;
    if (parse_table(buf.str(), x, &arch) && (arch.empty() || device_is(arch))) v = x;
    return v;
  }();
  return t;
}

std::string format_tune(const Tune& t, bool alloc) {
  char b[512];
  snprintf(b, sizeof(b),
           "rows_bpc=%d,rows_unroll=%d,cols_bpc=%d,cols_unroll=%d,qe_stage=%d,rows_stage=%d,brows_stage=%d,"
           "brows_unroll=%d,sym_wg=%d,sym_units=%d,bsym_units=%d,bsym_wave=%d,sym_teams=%d,sym_rows=%d,sym_pipe=%d,"
           "ld_nt=%d,upd_threads=%d,mv_rt=%d,cg_fold=%d",
           t.rows_bpc, t.rows_unroll, t.cols_bpc, t.cols_unroll, t.qe_stage, t.rows_stage, t.brows_stage,
           t.brows_unroll, t.sym_wg, t.sym_units, t.bsym_units, t.bsym_wave, t.sym_teams, t.sym_rows, t.sym_pipe,
           t.ld_nt, t.upd_threads, t.mv_rt, t.cg_fold);
  std::string s(b);
  if (alloc) {
    snprintf(b, sizeof(b), ",ld_pad=%d,op_t=%d,k0_sym=%d", t.ld_pad, t.op_t, t.k0_sym);
    s += b;
  }
  return s;
}

}  // namespace

Tune& tune() { return t_cur ? *const_cast<Tune*>(t_cur) : table().base; }

TuneScope::TuneScope(int n) : prev_(t_cur) {
  const TuneTable& t = table();
  const Tune* sel = &t.base;
  if (n > 0)
    for (auto& b : t.buckets)
      if (n <= b.first) {
        sel = &b.second;
        break;
      }
  t_cur = sel;
}

TuneScope::~TuneScope() { t_cur = prev_; }

}  // namespace qpg

extern "C" {

qp_status qp_tune_set(const char* spec) {
  if (!spec) return QP_E_INVALID;
  qpg::TuneTable t;
  if (!qpg::parse_table(spec, t, nullptr)) return QP_E_INVALID;
  qpg::TuneTable& cur = qpg::table();
  // the layout choices of existing contexts must not change under them
  if (t.base.ld_pad != cur.base.ld_pad || t.base.op_t != cur.base.op_t || t.base.k0_sym != cur.base.k0_sym)
    return QP_E_INVALID;
  cur = t;
  return QP_OK;
}

qp_status qp_tune_get(char* buf, size_t len, size_t* needed) {
  const qpg::TuneTable& t = qpg::table();
  std::string s = "default " + qpg::format_tune(t.base, true) + "\n";
  for (auto& b : t.buckets) s += "n<=" + std::to_string(b.first) + " " + qpg::format_tune(b.second, false) + "\n";
  if (needed) *needed = s.size() + 1;
  if (!buf) return QP_OK;
  if (len < s.size() + 1) return QP_E_INVALID;
  memcpy(buf, s.c_str(), s.size() + 1);
  return QP_OK;
}

}  // extern "C"

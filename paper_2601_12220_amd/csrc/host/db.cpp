#include "db.h"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <vector>

namespace bes {

int log_level() {
  const char *s = std::getenv("BES_LOG");
  return s ? std::atoi(s) : 0;
}

static std::vector<std::string> split(const std::string &s, char sep) {
  std::vector<std::string> r;
  std::string cur;
  for (char c : s) {
    if (c == sep) {
      r.push_back(cur);
      cur.clear();
    } else {
      cur += c;
    }
  }
  r.push_back(cur);
  return r;
}

static bool to_int(const std::string &s, int32_t &v) {
  if (s.empty()) return false;
  char *end = nullptr;
  long x = std::strtol(s.c_str(), &end, 10);
  if (*end != '\0') return false;
  v = (int32_t)x;
  return true;
}

bool TuningDB::parse_line(const std::string &line) {
  auto f = split(line, '\t');
  if (f.size() != 5 || f[0].empty() || f[1].empty()) return false;
  TuningRecord r;
  if (!to_int(f[2], r.cfg.template_id)) return false;
  if (r.cfg.template_id < BES_T_FEM_STREAM || r.cfg.template_id > BES_T_MFMA) return false;
  auto ps = split(f[3], ',');
  if (ps.size() != 6) return false;
  for (int k = 0; k < 6; ++k)
    if (!to_int(ps[k], r.cfg.p[k])) return false;
  char *end = nullptr;
  r.seconds = std::strtod(f[4].c_str(), &end);
  if (end == f[4].c_str() || *end != '\0') return false;
  recs_[{f[0], f[1]}] = r;
  return true;
}

int TuningDB::open(const char *path, std::string &err) {
  recs_.clear();
  skipped_ = 0;
  path_ = path ? path : "";
  if (path_.empty()) return BES_OK;
  std::ifstream in(path_);
  if (!in) return BES_OK;  // created on the first record
  std::string line;
  int64_t lineno = 0;
  while (std::getline(in, line)) {
    ++lineno;
    if (line.empty() || line[0] == '#') continue;
    if (!parse_line(line)) {
      ++skipped_;
      if (log_level() >= 1)
        std::fprintf(stderr, "bes: tuning db %s:%lld: skipping malformed record\n",
                     path_.c_str(), (long long)lineno);
    }
  }
  (void)err;
  return BES_OK;
}

const TuningRecord *TuningDB::find(const std::string &key, const std::string &arch) const {
  auto it = recs_.find({key, arch});
  return it == recs_.end() ? nullptr : &it->second;
}

int TuningDB::record(const std::string &key, const std::string &arch, const bes_config &cfg,
                     double seconds, std::string &err) {
  if (key.find('\t') != std::string::npos || key.find('\n') != std::string::npos ||
      arch.find('\t') != std::string::npos || arch.find('\n') != std::string::npos || key.empty() ||
      arch.empty()) {
    err = "key and arch must be non-empty and free of tabs and newlines";
    return BES_E_INVALID;
  }
  TuningRecord r;
  r.cfg = cfg;
  r.seconds = seconds;
  recs_[{key, arch}] = r;
  if (path_.empty()) return BES_OK;
  std::ofstream out(path_, std::ios::app);
  if (!out) {
    err = "cannot append to tuning db " + path_;
    return BES_E_INVALID;
  }
  std::ostringstream ps;
  for (int k = 0; k < 6; ++k) ps << (k ? "," : "") << cfg.p[k];
  char sec[64];
  std::snprintf(sec, sizeof sec, "%.9g", seconds);
  out << key << '\t' << arch << '\t' << cfg.template_id << '\t' << ps.str() << '\t' << sec << '\n';
  return BES_OK;
}

}  // namespace bes

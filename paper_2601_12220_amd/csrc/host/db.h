// Database of performance facts (Section "Integration of Optimized Batched
// Einsums into Practical Programs"): maps (canonical key, device arch) to the
// best known kernel configuration and its measured time.
//
// Storage: an append-only text file, one record per line,
//   <key> TAB <arch> TAB <template> TAB <p0,...,p5> TAB <seconds>
// The last record for a (key, arch) pair wins.  Malformed lines are skipped
// (with a warning on stderr when BES_LOG >= 1).
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <utility>

#include "../../../include/bes.h"

namespace bes {

struct TuningRecord {
  bes_config cfg{};
  double seconds = 0.0;
};

class TuningDB {
 public:
  int open(const char *path, std::string &err);
  const TuningRecord *find(const std::string &key, const std::string &arch) const;
  int record(const std::string &key, const std::string &arch, const bes_config &cfg,
             double seconds, std::string &err);
  size_t size() const { return recs_.size(); }
  int64_t skipped_lines() const { return skipped_; }

  int64_t hits = 0, misses = 0;

 private:
  bool parse_line(const std::string &line);
  std::string path_;
  std::map<std::pair<std::string, std::string>, TuningRecord> recs_;
  int64_t skipped_ = 0;
};

int log_level();

}  // namespace bes

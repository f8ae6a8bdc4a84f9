// Persistent autotuning results. The cache is a JSON object whose keys name a
// problem shape (or shape bucket) and whose values are objects of integer
// fields, written one entry per line, at the path given by the environment
// variable MX_TUNE_CACHE; with the variable unset nothing is read or written.
#pragma once
#include <map>
#include <string>

namespace mx {

using TuneFields = std::map<std::string, long long>;

// true when the variable is set and the file holds an entry for key
bool tune_cache_get(const std::string& key, TuneFields& out);
// adds or replaces the entry for key: the whole file is read, updated,
// written to a temporary file beside it and renamed into place, so a reader
// never sees a partial file (concurrent writers keep the last rename)
void tune_cache_put(const std::string& key, const TuneFields& fields);

}  // namespace mx

// Persisted split-K choices of mds_autotune.  With the environment variable
// MDS_TUNE_CACHE naming a file, mds_autotune records the splits it chose for
// a plan's key, and a later plan with the same key whose splits are all
// automatic starts from them.  One text line per key:
//   <arch> <cus> <form> <flags> <d_dtype> <n> <l_pad> <q> <range> <proj> <write> <f32>
// The file is rewritten whole through a temporary file and a rename, so a
// reader sees either the old or the new contents; concurrent writers keep
// the last record.  Host code only.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "mds_internal.h"

namespace mds {
namespace {

std::mutex g_cache_mutex;

const char* cache_path() {
  const char* p = getenv("MDS_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// key of the current device and the plan, or false without a device
bool make_key(const TuneKey& k, char* out, size_t size) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  char arch[64];
  snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
  for (char* c = arch; *c; ++c)
    if (*c == ' ' || *c == ':') *c = '_';  // one token (the name may carry target features)
  snprintf(out, size, "%s %d %d %d %d %lld %d %d", arch, prop.multiProcessorCount, k.form, k.flags, k.d_dtype,
           (long long)k.n, k.l_pad, k.q);
  return true;
}

// the key part of a line (its first 8 tokens) and the 4 splits after it
bool parse_line(const char* line, std::string& key, int (&splits)[4]) {
  char a[64];
  int cus, form, flags, dt, lp, q;
  long long n;
  if (sscanf(line, "%63s %d %d %d %d %lld %d %d %d %d %d %d", a, &cus, &form, &flags, &dt, &n, &lp, &q, &splits[0],
             &splits[1], &splits[2], &splits[3]) != 12)
    return false;
  char buf[160];
  snprintf(buf, sizeof(buf), "%s %d %d %d %d %lld %d %d", a, cus, form, flags, dt, n, lp, q);
  key = buf;
  return true;
}

}  // namespace

bool tune_cache_lookup(const TuneKey& k, int (&splits)[4]) {
  const char* path = cache_path();
  if (!path) return false;
  char key[160];
  if (!make_key(k, key, sizeof(key))) return false;
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    std::string lk;
    int s[4];
    if (parse_line(line, lk, s) && lk == key) {  // the last matching line wins
      for (int i = 0; i < 4; ++i) splits[i] = s[i];
      found = true;
    }
  }
  fclose(f);
  return found;
}

bool tune_cache_store(const TuneKey& k, const int (&splits)[4]) {
  const char* path = cache_path();
  if (!path) return false;
  char key[160];
  if (!make_key(k, key, sizeof(key))) return false;
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  std::vector<std::string> keep;
  if (FILE* f = fopen(path, "r")) {
    char line[256];
    while (fgets(line, sizeof(line), f)) {
      std::string lk;
      int s[4];
      if (parse_line(line, lk, s) && lk != key) keep.push_back(line);
    }
    fclose(f);
  }
  char rec[256];
  snprintf(rec, sizeof(rec), "%s %d %d %d %d\n", key, splits[0], splits[1], splits[2], splits[3]);
  keep.push_back(rec);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  bool ok = true;
  for (const std::string& l : keep) ok = ok && fputs(l.c_str(), f) >= 0;
  ok = (fclose(f) == 0) && ok;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace mds

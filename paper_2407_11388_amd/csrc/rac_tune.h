// Autotuner tables (tune.hip): the measured choice of path and work-item
// size per problem shape, looked up before a call and filled by measurement.
#pragma once

#include <stdint.h>

#include <string>

namespace rac {

enum { kTuneAuto = 0, kTuneRules = 1, kTuneMeasure = 2 };   // RAC_TUNE: (unset), rules, measure
enum { kTuneSingle = 0, kTuneBatch = 1 };                   // one state per call, many states
enum { kSourceRules = 0, kSourceShipped = 1, kSourceCache = 2, kSourceMeasured = 3 };

struct TuneChoice {
    int32_t path = 0;              // RAC_PATH_BITS / INT8 / MFMA
    int32_t item_scale_log2 = 0;   // work items of 2^s times the default size (bit / int8 rows)
    int32_t handoff = -1;          // matrix-core path: states left when the rest moves to the
                                   // bit rows (-1: the default)
    int32_t source = kSourceRules; // where the choice came from
    double ms = 0.0;               // its measured time per call
};

int tune_mode();
std::string tune_user_file();      // RAC_TUNE_CACHE, else ~/.cache/rac_tune_gfx950.txt
std::string tune_shipped_file();   // RAC_TUNE_TABLE, else rac_tune_gfx950.txt beside librac.so
// Key of a shape: kind, d, n (powers of 2 at least), density bucket (0.05, 0.1, 0.25,
// 0.5, 0.75, 1), states per call (power of 2 at least).
std::string tune_key(int kind, int32_t n, int32_t d, int64_t arcs, int32_t B);
bool tune_lookup(const std::string &key, TuneChoice *out);
void tune_store(const std::string &key, const TuneChoice &c);   // also appends to the user file
void tune_forget();                                              // drop the in-memory table

}  // namespace rac

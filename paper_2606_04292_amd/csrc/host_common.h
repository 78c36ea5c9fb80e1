// Host helpers shared by the single-grid API and the serving engine: error
// reporting, descriptor and law validation, the level hierarchy.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/richards.h"
#include "rs_internal.h"

namespace rs {

// Record a thread-local error message (rs_last_error) and return code.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIPCALL(x)                                                                     \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) return fail(RS_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int validate_desc(const rs_grid_desc *d);
int validate_law(const rs_constitutive *c);
// Levels down to 3 nodes on the shortest axis.
int level_count(const rs_grid_desc *d);
Geo make_geo(const rs_grid_desc *d, int lev);
Law make_law(const rs_constitutive *c);
long long count_unknowns(const Geo &g);

}  // namespace rs

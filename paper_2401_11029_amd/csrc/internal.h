// internal.h -- host-side types shared by the library's translation units.
#pragma once

#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cflr.h"

namespace cflr {

// Error carrying a cflr_status; converted at the C boundary.
struct Error : std::runtime_error {
    cflr_status status;
    Error(cflr_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

// A grammar lowered to strict weak Chomsky normal form (Definition 1):
// every production is x -> eps, x -> t (t a terminal) or x -> y z with y, z
// non-terminals.  Matrices 0..user-1 are the text's non-terminals; after
// them come wrappers T_t for terminals that stood in binary positions.
struct Lowered {
    std::vector<std::string> user_names;       // first-appearance order
    std::vector<std::string> mat_names;        // user names, then "<t>" wrappers and
                                               // "<y ... z>" suffix helpers
    std::vector<std::string> terminals;        // distinct terminal names
    struct Bin { uint32_t c, a, b; };
    std::vector<Bin> binary;                   // deduplicated
    std::vector<std::pair<uint32_t, uint32_t>> term;  // (terminal index, matrix)
    std::vector<uint32_t> eps;                 // matrices with x -> eps
    // per matrix: receives pairs from binary productions / used in slot a
    // (needs the column-major copy) / used in slot b (row-major copy)
    std::vector<uint8_t> dynamic, slot_a, slot_b;
    uint32_t wrappers = 0, helpers = 0;
    uint32_t nmat() const { return (uint32_t)mat_names.size(); }
};

Lowered parse_and_lower(const char *text, size_t len);

}  // namespace cflr

struct cflr_grammar {
    cflr::Lowered low;
    uint64_t serial;  // identity for caches keyed by grammar
};

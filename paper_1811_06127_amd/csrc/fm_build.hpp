// fm_build.hpp -- host-side index construction and file I/O.
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/fm.h"

namespace fm {

constexpr uint32_t kSaSample = 32;   // SA values kept for locating: rows that are multiples of 32 (Eq. 4-5)

struct HostSide {                 // one text's packed BWT and its constants
    std::vector<uint32_t> words;  // 2-bit codes, '$' stored as 0
    uint64_t dollar = 0;
    uint64_t C[5] = {0, 0, 0, 0, 0};
    const uint32_t *dev_words = nullptr;   // the same words already in device memory (then `words` is empty)
    std::vector<uint32_t> samples;         // SA values of rows 0, 32, 64, ... (locating), if built
    const uint32_t *dev_samples = nullptr; // the same in device memory
};

int build_bwt(const uint8_t *text, uint64_t n, uint8_t *bwt, uint64_t *dollar_row,
              std::vector<uint32_t> *samples = nullptr);
int pack_codes(const uint8_t *codes, uint64_t count, uint32_t *words, uint64_t dollar_row);
int bwt_stats(const uint8_t *bwt, uint64_t rows, uint64_t *dollar_row, uint64_t C[5]);
int build_side(const uint8_t *text, uint64_t n, bool reverse, HostSide &out, bool want_samples = false);
int write_index_file(const char *path, uint64_t n, const HostSide &fwd, const HostSide *rev);
int read_index_file(const char *path, bool want_rev, uint64_t *n, HostSide &fwd, HostSide &rev, bool *has_rev);
// n and whether a reverse index is present, from the header alone (checked as by read_index_file).
int read_index_header(const char *path, uint64_t *n, bool *has_rev);

}  // namespace fm

// build.cpp -- the library's index builder (host): suffix array of R$ by induced sorting
// (SA-IS: Nong, Zhang and Chan, "Two efficient algorithms for linear time suffix array
// construction", IEEE TC 2011), the BWT from it (Eq. 2), C (Background), 2-bit packing,
// and the index file format. Index construction is a one-off step before searching,
// like `bwa index`; nothing here runs on the search path.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "fm_build.hpp"

namespace fm {
namespace {

// Suffix array of T[0..n) where T[n-1] is a unique smallest sentinel and symbols are in
// [0, K). Idx is a signed integer type able to hold n.
template <typename Idx, typename Sym>
void sais(const Sym *T, Idx *SA, Idx n, Idx K)
{
    if (n == 1) {
        SA[0] = 0;
        return;
    }
    std::vector<uint8_t> stype(n);   // 1: S-type suffix, 0: L-type
    stype[n - 1] = 1;
    for (Idx i = n - 2; i >= 0; --i)
        stype[i] = (T[i] < T[i + 1] || (T[i] == T[i + 1] && stype[i + 1])) ? 1 : 0;
    auto is_lms = [&](Idx i) { return i > 0 && stype[i] && !stype[i - 1]; };
    std::vector<Idx> bkt(K);
    auto buckets = [&](bool ends) {
        std::fill(bkt.begin(), bkt.end(), (Idx)0);
        for (Idx i = 0; i < n; ++i) bkt[T[i]]++;
        Idx s = 0;
        for (Idx c = 0; c < K; ++c) {
            s += bkt[c];
            bkt[c] = ends ? s : s - bkt[c];
        }
    };
    auto induce = [&]() {
        buckets(false);   // L-type suffixes, left to right from bucket starts
        for (Idx i = 0; i < n; ++i) {
            const Idx j = SA[i] - 1;
            if (SA[i] > 0 && !stype[j]) SA[bkt[T[j]]++] = j;
        }
        buckets(true);    // S-type suffixes, right to left from bucket ends
        for (Idx i = n - 1; i >= 0; --i) {
            const Idx j = SA[i] - 1;
            if (SA[i] > 0 && stype[j]) SA[--bkt[T[j]]] = j;
        }
    };
    // 1. sort the LMS substrings by one round of induced sorting
    buckets(true);
    std::fill(SA, SA + n, (Idx)-1);
    for (Idx i = 1; i < n; ++i)
        if (is_lms(i)) SA[--bkt[T[i]]] = i;
    induce();
    Idx n1 = 0;
    for (Idx i = 0; i < n; ++i)
        if (is_lms(SA[i])) SA[n1++] = SA[i];
    // 2. name them; equal names for equal LMS substrings
    std::fill(SA + n1, SA + n, (Idx)-1);
    Idx name = 0, prev = -1;
    for (Idx i = 0; i < n1; ++i) {
        const Idx pos = SA[i];
        bool diff = false;
        for (Idx d = 0; d < n; ++d) {
            if (prev == -1 || T[pos + d] != T[prev + d] || stype[pos + d] != stype[prev + d]) {
                diff = true;
                break;
            }
            if (d > 0 && (is_lms(pos + d) || is_lms(prev + d))) break;
        }
        if (diff) {
            ++name;
            prev = pos;
        }
        SA[n1 + pos / 2] = name - 1;
    }
    for (Idx i = n - 1, j = n - 1; i >= n1; --i)
        if (SA[i] >= 0) SA[j--] = SA[i];
    // 3. order of the LMS suffixes: directly if names are unique, else recursively
    Idx *SA1 = SA, *s1 = SA + n - n1;
    if (name < n1) sais<Idx, Idx>(s1, SA1, n1, name);
    else
        for (Idx i = 0; i < n1; ++i) SA1[s1[i]] = i;
    // 4. induce the full order from the sorted LMS suffixes
    buckets(true);
    for (Idx i = 1, j = 0; i < n; ++i)
        if (is_lms(i)) s1[j++] = i;
    for (Idx i = 0; i < n1; ++i) SA1[i] = s1[SA1[i]];
    std::fill(SA + n1, SA + n, (Idx)-1);
    for (Idx i = n1 - 1; i >= 0; --i) {
        const Idx j = SA[i];
        SA[i] = -1;
        SA[--bkt[T[j]]] = j;
    }
    induce();
}

template <typename Idx>
int bwt_with(const uint8_t *text, uint64_t n, uint8_t *bwt, uint64_t *dollar_row, std::vector<uint32_t> *samples)
{
    const Idx N = (Idx)(n + 1);
    std::vector<uint8_t> T;
    std::vector<Idx> SA;
    try {
        T.resize(n + 1);
        SA.resize(n + 1);
    } catch (const std::bad_alloc &) {
        return FM_ENOMEM;
    }
    for (uint64_t i = 0; i < n; ++i) T[i] = (uint8_t)(text[i] + 1);   // '$' = 0 below every base
    T[n] = 0;
    sais<Idx, uint8_t>(T.data(), SA.data(), N, (Idx)5);
    if (samples) {
        try {
            samples->resize((n + 1 + kSaSample - 1) / kSaSample);
        } catch (const std::bad_alloc &) {
            return FM_ENOMEM;
        }
        for (uint64_t j = 0; j < samples->size(); ++j) (*samples)[j] = (uint32_t)SA[j * kSaSample];
    }
    for (uint64_t i = 0; i <= n; ++i) {
        const Idx s = SA[i];
        if (s > 0) {
            bwt[i] = text[s - 1];
        } else {
            bwt[i] = 4;
            *dollar_row = i;
        }
    }
    return FM_OK;
}

uint64_t fnv1a(const void *p, size_t bytes, uint64_t h)
{
    const uint8_t *b = (const uint8_t *)p;
    for (size_t i = 0; i < bytes; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

constexpr char kMagic[8] = {'F', 'M', 'O', 'C', 'C', '0', '0', '2'};

struct FileHeader {
    char magic[8];
    uint64_t n, flags, dollar, C[5], rev_dollar, rev_C[5], words, checksum;
};

// FNV-1a over the header (checksum field zero) and then the packed words of each side.
uint64_t file_checksum(const FileHeader &h, const uint32_t *fwd, const uint32_t *rev)
{
    FileHeader z = h;
    z.checksum = 0;
    uint64_t sum = fnv1a(&z, sizeof z, 0xcbf29ce484222325ull);
    sum = fnv1a(fwd, h.words * 4, sum);
    if (rev) sum = fnv1a(rev, h.words * 4, sum);
    return sum;
}

// The header's C and '$' row agree with the packed words of rows 0..n: C[c+1] - C[c] is
// the number of rows holding code c, less the '$' row for code 0 (it is stored as 0),
// and the word at the '$' row holds 0 there.
bool side_consistent(const uint32_t *words, uint64_t n, uint64_t dollar, const uint64_t C[5])
{
    if (dollar > n || C[0] != 0 || C[4] != n) return false;
    if ((words[dollar / 16] >> (2 * (dollar % 16))) & 3u) return false;
    uint64_t cnt[4] = {0, 0, 0, 0};
    const uint64_t rows = n + 1, full = rows / 16;
    for (uint64_t w = 0; w < full; ++w) {
        const uint32_t x = words[w], lo = x & 0x55555555u, hi = (x >> 1) & 0x55555555u;
        const uint32_t t = (uint32_t)__builtin_popcount(lo & hi);
        cnt[3] += t;
        cnt[2] += (uint32_t)__builtin_popcount(hi) - t;
        cnt[1] += (uint32_t)__builtin_popcount(lo) - t;
    }
    for (uint64_t r = full * 16; r < rows; ++r) {
        const uint32_t c = (words[r / 16] >> (2 * (r % 16))) & 3u;
        if (c) cnt[c]++;
    }
    if (rows % 16 && (words[full] >> (2 * (rows % 16))) != 0) return false;   // unused bits stay 0
    cnt[0] = rows - cnt[1] - cnt[2] - cnt[3] - 1;
    for (int c = 0; c < 4; ++c)
        if (C[c] > C[c + 1] || C[c + 1] - C[c] != cnt[c]) return false;
    return true;
}

// Reads and checks the header: magic, sizes, flags.
int read_header(FILE *f, FileHeader &h)
{
    if (fread(&h, sizeof h, 1, f) != 1) return FM_EFORMAT;
    if (memcmp(h.magic, kMagic, 8) != 0) return FM_EFORMAT;
    if (h.n + 1 >= (1ull << 32) || h.words != (h.n + 1 + 15) / 16 || (h.flags & ~(uint64_t)FM_LOAD_REVERSE))
        return FM_EFORMAT;
    return FM_OK;
}

}  // namespace

int build_bwt(const uint8_t *text, uint64_t n, uint8_t *bwt, uint64_t *dollar_row, std::vector<uint32_t> *samples)
{
    if (n + 1 >= (1ull << 32)) return FM_ERANGE;
    for (uint64_t i = 0; i < n; ++i)
        if (text[i] > 3) return FM_EINVAL;
    if (n + 1 < (1ull << 31) - 1) return bwt_with<int32_t>(text, n, bwt, dollar_row, samples);
    return bwt_with<int64_t>(text, n, bwt, dollar_row, samples);
}

int pack_codes(const uint8_t *codes, uint64_t count, uint32_t *words, uint64_t dollar_row)
{
    const uint64_t nw = (count + 15) / 16;
    memset(words, 0, nw * 4);
    for (uint64_t i = 0; i < count; ++i) {
        uint32_t c = codes[i];
        if (i == dollar_row) c = 0;                 // '$' is stored as code 0
        else if (c > 3) return FM_EINVAL;
        words[i / 16] |= c << (2 * (i % 16));
    }
    return FM_OK;
}

int bwt_stats(const uint8_t *bwt, uint64_t rows, uint64_t *dollar_row, uint64_t C[5])
{
    uint64_t cnt[5] = {0, 0, 0, 0, 0};
    uint64_t dr = ~0ull;
    for (uint64_t i = 0; i < rows; ++i) {
        const uint8_t c = bwt[i];
        if (c > 4) return FM_EFORMAT;
        if (c == 4) dr = i;
        cnt[c]++;
    }
    if (cnt[4] != 1) return FM_EFORMAT;
    *dollar_row = dr;
    C[0] = 0;
    for (int c = 0; c < 4; ++c) C[c + 1] = C[c] + cnt[c];
    return FM_OK;
}

int build_side(const uint8_t *text, uint64_t n, bool reverse, HostSide &out, bool want_samples)
{
    std::vector<uint8_t> rtext;
    const uint8_t *src = text;
    if (reverse) {
        try {
            rtext.assign(text, text + n);
        } catch (const std::bad_alloc &) {
            return FM_ENOMEM;
        }
        std::reverse(rtext.begin(), rtext.end());
        src = rtext.data();
    }
    std::vector<uint8_t> bwt;
    try {
        bwt.resize(n + 1);
        out.words.assign((n + 1 + 15) / 16, 0u);
    } catch (const std::bad_alloc &) {
        return FM_ENOMEM;
    }
    int st = build_bwt(src, n, bwt.data(), &out.dollar, want_samples ? &out.samples : nullptr);
    if (st) return st;
    st = bwt_stats(bwt.data(), n + 1, &out.dollar, out.C);
    if (st) return st;
    return pack_codes(bwt.data(), n + 1, out.words.data(), out.dollar);
}

int write_index_file(const char *path, uint64_t n, const HostSide &fwd, const HostSide *rev)
{
    FileHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, kMagic, 8);
    h.n = n;
    h.flags = rev ? FM_LOAD_REVERSE : 0;
    h.dollar = fwd.dollar;
    memcpy(h.C, fwd.C, sizeof h.C);
    if (rev) {
        h.rev_dollar = rev->dollar;
        memcpy(h.rev_C, rev->C, sizeof h.rev_C);
    }
    h.words = fwd.words.size();
    h.checksum = file_checksum(h, fwd.words.data(), rev ? rev->words.data() : nullptr);
    FILE *f = fopen(path, "wb");
    if (!f) return FM_EIO;
    bool ok = fwrite(&h, sizeof h, 1, f) == 1;
    ok = ok && fwrite(fwd.words.data(), 4, fwd.words.size(), f) == fwd.words.size();
    if (rev) ok = ok && fwrite(rev->words.data(), 4, rev->words.size(), f) == rev->words.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? FM_OK : FM_EIO;
}

int read_index_header(const char *path, uint64_t *n, bool *has_rev)
{
    FILE *f = fopen(path, "rb");
    if (!f) return FM_EIO;
    FileHeader h;
    const int st = read_header(f, h);
    fclose(f);
    if (st) return st;
    *n = h.n;
    *has_rev = (h.flags & FM_LOAD_REVERSE) != 0;
    return FM_OK;
}

int read_index_file(const char *path, bool want_rev, uint64_t *n, HostSide &fwd, HostSide &rev, bool *has_rev)
{
    FILE *f = fopen(path, "rb");
    if (!f) return FM_EIO;
    FileHeader h;
    int st = read_header(f, h);
    const bool file_rev = !st && (h.flags & FM_LOAD_REVERSE);
    if (!st && want_rev && !file_rev) st = FM_EINVAL;
    if (!st) {
        try {
            fwd.words.resize(h.words);
            if (file_rev) rev.words.resize(h.words);
        } catch (const std::bad_alloc &) {
            st = FM_ENOMEM;
        }
    }
    if (!st && fread(fwd.words.data(), 4, h.words, f) != h.words) st = FM_EFORMAT;
    if (!st && file_rev && fread(rev.words.data(), 4, h.words, f) != h.words) st = FM_EFORMAT;
    if (!st && fgetc(f) != EOF) st = FM_EFORMAT;                  // nothing may follow the body
    fclose(f);
    if (st) return st;
    if (file_checksum(h, fwd.words.data(), file_rev ? rev.words.data() : nullptr) != h.checksum) return FM_EFORMAT;
    if (!side_consistent(fwd.words.data(), h.n, h.dollar, h.C)) return FM_EFORMAT;
    if (file_rev && !side_consistent(rev.words.data(), h.n, h.rev_dollar, h.rev_C)) return FM_EFORMAT;
    *n = h.n;
    fwd.dollar = h.dollar;
    memcpy(fwd.C, h.C, sizeof h.C);
    rev.dollar = h.rev_dollar;
    memcpy(rev.C, h.rev_C, sizeof h.rev_C);
    *has_rev = file_rev;
    return FM_OK;
}

}  // namespace fm

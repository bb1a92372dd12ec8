// Host-only driver of the graph compiler and the bundle reader, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host side by
// tests/test_host_sanitizers.py (no device code runs).  It compiles bundles of
// every algebra, reads them back with full validation, and feeds the reader
// corrupted copies: every case must end in the expected status without a
// sanitizer report.  Exit status 0 = all cases as expected.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../paper_2609_14831_amd/csrc/internal.h"

namespace cut {
static char g_msg[512];
void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
}
}  // namespace cut

using namespace cut;

static int failures = 0;

static int read_status(const std::string& path, bool verify) {
    try {
        HostGraph hg;
        read_bundle(path.c_str(), verify, hg);
        return CUT_OK;
    } catch (const Fail& f) {
        return f.st;
    }
}

static void expect(bool ok, const char* what, const std::string& path) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s): %s\n", what, path.c_str(), g_msg);
        ++failures;
    }
}

static std::vector<unsigned char> slurp(const std::string& p) {
    std::vector<unsigned char> d;
    FILE* f = std::fopen(p.c_str(), "rb");
    if (!f) return d;
    unsigned char buf[1 << 16];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) d.insert(d.end(), buf, buf + n);
    std::fclose(f);
    return d;
}

static void spit(const std::string& p, const std::vector<unsigned char>& d, size_t n) {
    FILE* f = std::fopen(p.c_str(), "wb");
    std::fwrite(d.data(), 1, n, f);
    std::fclose(f);
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    const std::string dir = argv[1];
    struct Case {
        int alg, size;
        unsigned flags;
    };
    const Case cases[] = {{CUT_ALG_EPQ, 4, 0}, {CUT_ALG_EPQ, 8, 0}, {CUT_ALG_MAJORANA, 8, 0},
                          {CUT_ALG_MAJORANA, 12, CUT_BUILD_OUTSIDE}, {CUT_ALG_MAJORANA, 16, 0},
                          {CUT_ALG_PAULI_BOSON, 256 * 1 + 3, CUT_BUILD_OUTSIDE},
                          {CUT_ALG_PAULI_BOSON, 256 * 2 + 2, 0}};
    int k = 0;
    for (const Case& c : cases) {
        const std::string p = dir + "/b" + std::to_string(k++) + ".cgb";
        cut_graph_desc d{};
        const cut_status st = cut_graph_build(c.alg, c.size, p.c_str(), 2, c.flags, &d);
        expect(st == CUT_OK, "build", p);
        if (st != CUT_OK) continue;
        expect(read_status(p, true) == CUT_OK, "read back", p);
        std::vector<unsigned char> raw = slurp(p);
        // a header byte, a section-table byte, then the first, middle and last
        // byte of every section (the alignment padding between sections
        // carries no data and no checksum), and truncations
        const size_t n = raw.size();
        BundleHeader h;
        std::memcpy(&h, raw.data(), sizeof h);
        std::vector<size_t> spots = {100, sizeof(BundleHeader) + 7};
        for (uint32_t q = 0; q < h.n_sections; ++q) {
            SectionEntry e;
            std::memcpy(&e, raw.data() + sizeof h + q * sizeof e, sizeof e);
            const uint64_t bytes = e.count * e.elem_bytes;
            if (bytes == 0) continue;
            for (uint64_t at : {e.offset, e.offset + bytes / 2, e.offset + bytes - 1}) spots.push_back((size_t)at);
        }
        for (size_t pos : spots) {
            std::vector<unsigned char> bad = raw;
            bad[pos] ^= 0x5A;
            const std::string q = p + ".bad";
            spit(q, bad, n);
            expect(read_status(q, true) != CUT_OK,
                   ("corrupt byte rejected at " + std::to_string(pos) + " of " + std::to_string(n)).c_str(), q);
            read_status(q, false);   // bounds checks alone: any status, no sanitizer report
        }
        for (size_t cut : {size_t(0), size_t(64), sizeof(BundleHeader) + 40, n / 2, n - 1}) {
            const std::string q = p + ".short";
            spit(q, raw, cut);
            expect(read_status(q, true) != CUT_OK, "truncated file rejected", q);
        }
    }
    // argument errors of the compiler
    expect(cut_graph_build(CUT_ALG_MAJORANA, 7, (dir + "/x.cgb").c_str(), 1, 0, nullptr) == CUT_E_INVAL, "odd m",
           dir);
    expect(cut_graph_build(CUT_ALG_EPQ, 4, (dir + "/x.cgb").c_str(), 1, CUT_BUILD_OUTSIDE, nullptr) == CUT_E_INVAL,
           "outside with a closed registry", dir);
    expect(read_status(dir + "/does_not_exist", true) == CUT_E_IO, "missing file", dir);
    std::printf("%d failures\n", failures);
    return failures == 0 ? 0 : 1;
}

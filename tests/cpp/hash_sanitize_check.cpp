// Sanitizer run of the two host-side hashing codes: the CPU oracle (oracle/hash_oracle.c)
// and the library's host share of a CPU + GPU split (hb_cpu.cpp).  Every message sits in a
// heap buffer of exactly its length, so the address sanitizer flags any read past its end
// (or before its start); the undefined-behaviour sanitizer flags shifts by 32, signed
// overflow and misaligned loads.  Lengths 0..300 (every residue mod 64, up to five blocks)
// and 1 MiB-class messages, all three algorithms; the two codes must also agree.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

extern "C" int oracle_hash(int algo, const uint8_t *msg, uint64_t len, uint8_t *out);

namespace hb {
void cpu_hash_range(const uint8_t *algos, int algo, const uint8_t *msgs, const uint64_t *offs, const uint64_t *lens,
                    uint64_t i0, uint64_t i1, uint8_t *out, uint32_t stride, int threads);
// the two library helpers hb_cpu.cpp's C entry point refers to (not exercised here)
int set_error(int status, const std::string &) { return status; }
int digest_size(int algo) { return algo == 0 ? 16 : algo == 1 ? 20 : algo == 2 ? 32 : 0; }
}  // namespace hb

namespace {

uint64_t g_state = 0x2407093330000001ull;
uint8_t next_byte()
{
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return uint8_t(g_state >> 56);
}

int check(int algo, uint64_t len, uint64_t shift)
{
    // an exact-size allocation, the message starting `shift` bytes into it
    uint8_t *buf = static_cast<uint8_t *>(std::malloc(len + shift ? len + shift : 1));
    for (uint64_t i = 0; i < len + shift; ++i) buf[i] = next_byte();
    const uint8_t *msg = buf + shift;
    uint8_t want[32] = {0}, got[32];
    std::memset(got, 0xEE, sizeof got);
    if (oracle_hash(algo, msg, len, want) != 0) {
        std::free(buf);
        std::printf("oracle failed: algo %d len %llu\n", algo, (unsigned long long)len);
        return 1;
    }
    const uint64_t off = 0;
    hb::cpu_hash_range(nullptr, algo, msg, &off, &len, 0, 1, got, 32u, 1);
    std::free(buf);
    const int ds = hb::digest_size(algo);
    if (std::memcmp(want, got, size_t(ds)) != 0) {
        std::printf("digests differ: algo %d len %llu shift %llu\n", algo, (unsigned long long)len,
                    (unsigned long long)shift);
        return 1;
    }
    for (int q = ds; q < 32; ++q)
        if (got[q] != 0) {
            std::printf("slot not zero-filled: algo %d len %llu\n", algo, (unsigned long long)len);
            return 1;
        }
    return 0;
}

}  // namespace

int main()
{
    int bad = 0, runs = 0;
    for (int algo = 0; algo < 3; ++algo) {
        for (uint64_t len = 0; len <= 300; ++len, ++runs) bad += check(algo, len, len % 5);
        const uint64_t big[] = {1ull << 20, (1ull << 20) + 55, (1ull << 20) + 56, (1ull << 20) + 63,
                                (1ull << 20) + 119, 3 * (1ull << 19) + 1};
        for (uint64_t len : big) { bad += check(algo, len, 3); ++runs; }
    }
    if (bad) {
        std::printf("%d of %d cases failed\n", bad, runs);
        return 1;
    }
    std::printf("sanitized hashing ok: %d cases\n", runs);
    return 0;
}

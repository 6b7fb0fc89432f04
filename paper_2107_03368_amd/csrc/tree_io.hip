// Saving and loading a Dissimilarity Tree (Section 4.1: the index is built
// once, offline, and then queried).
//
// A file holds the tree's structure and its rows, nothing derived:
//   header, 64 bytes (all integers little-endian):
//     0  magic "QDTREE\0\0"        8  uint32 version (1)
//     12 uint32 flags (bit 0: product images, bit 1: popcount ranges)
//     16 uint64 n (rows)           24 uint64 n_nodes
//     32 uint32 max_leaf           36 uint32 reserved (0)
//     40 uint64 payload bytes      48 uint64 payload hash
//     56 uint64 header hash (of bytes 0..55)
//   payload, each section zero-padded to a multiple of 8 bytes:
//     rows   n x 64 uint64, in leaf order
//     perm   n uint32: database row of each leaf-order position
//     child  n_nodes x 2 int32: similar, dissimilar child (-1, -1 for a leaf)
//     begin  n_nodes uint32, count n_nodes uint32
// Hashes are FNV-1a over 64-bit little-endian words (offset basis
// 0xcbf29ce484222325, prime 0x100000001b3).  Loading checks the header, both
// hashes and the structure (breadth-first numbering with children in parent
// order, children splitting their parent's rows, a permutation) on the host
// before any device work, then recomputes every derived array (images,
// popcounts and their ranges, parents, levels, inverse permutation, block
// images) from the rows, so a loaded tree is an exact index of its rows.
#include <stdio.h>
#include <string.h>

#include <vector>

#include "qd_internal.h"
#include "qd_tree.h"

namespace qd {
namespace {

constexpr char kMagic[8] = {'Q', 'D', 'T', 'R', 'E', 'E', 0, 0};
constexpr uint32_t kVersion = 1;
constexpr size_t kHeader = 64;
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull, kFnvPrime = 0x100000001b3ull;
constexpr size_t kChunk = 64ull << 20;  // bytes per read or write

struct Header {
    char magic[8];
    uint32_t version, flags;
    uint64_t n, n_nodes;
    uint32_t max_leaf, reserved;
    uint64_t payload, payload_hash, header_hash;
};
static_assert(sizeof(Header) == kHeader, "header layout");

uint64_t fnv(uint64_t h, const void *data, size_t bytes) {  // bytes: a multiple of 8
    const unsigned char *p = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < bytes; i += 8) {
        uint64_t w;
        memcpy(&w, p + i, 8);
        h = (h ^ w) * kFnvPrime;
    }
    return h;
}

inline uint64_t pad8(uint64_t b) { return (b + 7) / 8 * 8; }

uint64_t payload_bytes(uint64_t n, uint64_t nn) {
    return n * 512 + pad8(n * 4) + nn * 8 + 2 * pad8(nn * 4);
}

struct File {
    FILE *f = nullptr;
    ~File() {
        if (f) fclose(f);
    }
};

// Reads `bytes` into dst (if not null), hashing them.
bool read_hash(FILE *f, void *dst, uint64_t bytes, uint64_t &h, std::vector<unsigned char> &buf) {
    unsigned char *out = static_cast<unsigned char *>(dst);
    while (bytes) {
        const size_t m = (size_t)std::min<uint64_t>(bytes, kChunk);
        unsigned char *at = out ? out : buf.data();
        if (fread(at, 1, m, f) != m) return false;
        h = fnv(h, at, m);
        if (out) out += m;
        bytes -= m;
    }
    return true;
}

}  // namespace
}  // namespace qd

extern "C" int qd_tree_save(qd_tree_t t, const char *path) {
    using namespace qd;
    if (!t || !path) return fail(QD_ERR_INVALID, "null argument");
    (void)hipSetDevice(t->device);
    const uint64_t n = t->n, nn = t->n_nodes;
    File file;
    file.f = fopen(path, "wb");
    if (!file.f) return fail(QD_ERR_IO, "cannot open %s for writing", path);
    Header hd;
    memset(&hd, 0, sizeof hd);
    if (fwrite(&hd, 1, kHeader, file.f) != kHeader) return fail(QD_ERR_IO, "write failed: %s", path);
    uint64_t h = kFnvBasis;
    std::vector<unsigned char> buf(kChunk);
    auto put = [&](const void *dev, uint64_t bytes) -> int {
        const unsigned char *src = static_cast<const unsigned char *>(dev);
        const uint64_t total = pad8(bytes);
        for (uint64_t o = 0; o < total; o += kChunk) {
            const size_t m = (size_t)std::min<uint64_t>(total - o, kChunk);
            const size_t real = (size_t)(o + m <= bytes ? m : bytes > o ? bytes - o : 0);
            memset(buf.data() + real, 0, m - real);
            if (real) QD_HIP_CHECK(hipMemcpy(buf.data(), src + o, real, hipMemcpyDeviceToHost));
            h = fnv(h, buf.data(), m);
            if (fwrite(buf.data(), 1, m, file.f) != m) return fail(QD_ERR_IO, "write failed: %s", path);
        }
        return QD_OK;
    };
    int rc;
    if ((rc = put(t->d_sorted, n * 512)) != QD_OK || (rc = put(t->d_perm, n * 4)) != QD_OK ||
        (rc = put(t->d_child, nn * 8)) != QD_OK || (rc = put(t->d_begin, nn * 4)) != QD_OK ||
        (rc = put(t->d_count, nn * 4)) != QD_OK)
        return rc;
    memcpy(hd.magic, kMagic, 8);
    hd.version = kVersion;
    hd.flags = (t->has_and ? 1u : 0u) | (t->d_pmin ? 2u : 0u);
    hd.n = n;
    hd.n_nodes = nn;
    hd.max_leaf = t->max_leaf;
    hd.payload = payload_bytes(n, nn);
    hd.payload_hash = h;
    hd.header_hash = fnv(kFnvBasis, &hd, kHeader - 8);
    if (fseek(file.f, 0, SEEK_SET) != 0 || fwrite(&hd, 1, kHeader, file.f) != kHeader)
        return fail(QD_ERR_IO, "write failed: %s", path);
    if (fclose(file.f) != 0) {
        file.f = nullptr;
        return fail(QD_ERR_IO, "write failed: %s", path);
    }
    file.f = nullptr;
    return QD_OK;
}

extern "C" int qd_tree_load(const char *path, void *stream, qd_tree_t *out) {
    using namespace qd;
    if (!path || !out) return fail(QD_ERR_INVALID, "null argument");
    *out = nullptr;
    File file;
    file.f = fopen(path, "rb");
    if (!file.f) return fail(QD_ERR_IO, "cannot open %s", path);
    FILE *f = file.f;
    Header hd;
    if (fread(&hd, 1, kHeader, f) != kHeader) return fail(QD_ERR_FORMAT, "%s: shorter than a tree header", path);
    if (memcmp(hd.magic, kMagic, 8) != 0) return fail(QD_ERR_FORMAT, "%s: not a tree file", path);
    if (fnv(kFnvBasis, &hd, kHeader - 8) != hd.header_hash) return fail(QD_ERR_FORMAT, "%s: header hash mismatch", path);
    if (hd.version != kVersion) return fail(QD_ERR_FORMAT, "%s: version %u, this library reads %u", path, hd.version,
                                            kVersion);
    const uint64_t n = hd.n, nn = hd.n_nodes;
    if (n < 1 || n > QD_MAX_ROWS || nn < 1 || nn > 2 * n - 1 || hd.max_leaf < 1 || (hd.flags & ~3u) ||
        hd.reserved != 0 || hd.payload != payload_bytes(n, nn))
        return fail(QD_ERR_FORMAT, "%s: inconsistent header", path);
    if (fseek(f, 0, SEEK_END) != 0) return fail(QD_ERR_IO, "%s: seek failed", path);
    const long long size = ftell(f);
    if (size < 0 || (uint64_t)size != kHeader + hd.payload)
        return fail(QD_ERR_FORMAT, "%s: %lld bytes, the header says %llu", path, size,
                    (unsigned long long)(kHeader + hd.payload));
    if (fseek(f, (long)kHeader, SEEK_SET) != 0) return fail(QD_ERR_IO, "%s: seek failed", path);
    // pass 1, host only: hash everything, keep the structure
    std::vector<unsigned char> buf(kChunk);
    std::vector<uint32_t> perm(n), begin(nn), count(nn);
    std::vector<int32_t> child(2 * nn);
    uint64_t h = kFnvBasis;
    auto section = [&](void *dst, uint64_t bytes) {
        const uint64_t total = pad8(bytes);
        if (!read_hash(f, dst, bytes - bytes % 8, h, buf)) return false;
        if (total == bytes) return true;
        unsigned char last[8] = {0};
        if (fread(last, 1, 8, f) != 8) return false;
        const uint64_t keep = bytes % 8;
        for (uint64_t i = keep; i < 8; i++)
            if (last[i]) return false;  // padding must be zero
        if (dst) memcpy(static_cast<unsigned char *>(dst) + (bytes - keep), last, keep);
        h = fnv(h, last, 8);
        return true;
    };
    const bool rows_ok = section(nullptr, n * 512);
    const uint64_t h_rows = h;  // the rows are read again below: they must not change in between
    if (!rows_ok || !section(perm.data(), n * 4) || !section(child.data(), nn * 8) ||
        !section(begin.data(), nn * 4) || !section(count.data(), nn * 4))
        return fail(QD_ERR_FORMAT, "%s: truncated payload or non-zero padding", path);
    if (h != hd.payload_hash) return fail(QD_ERR_FORMAT, "%s: payload hash mismatch", path);
    // structure: breadth-first numbering, children split their parent's rows
    if (begin[0] != 0 || count[0] != n) return fail(QD_ERR_FORMAT, "%s: the root does not hold every row", path);
    uint64_t next = 1;
    for (uint64_t i = 0; i < nn; i++) {
        const int32_t a = child[2 * i], b = child[2 * i + 1];
        if (a < 0 && b < 0) continue;
        if ((uint64_t)a != next || (uint64_t)b != next + 1 || next + 1 >= nn)
            return fail(QD_ERR_FORMAT, "%s: node %llu: children not in breadth-first order", path,
                        (unsigned long long)i);
        next += 2;
        if (count[a] < 1 || count[b] < 1 || (uint64_t)count[a] + count[b] != count[i] || begin[a] != begin[i] ||
            begin[b] != begin[i] + count[a])
            return fail(QD_ERR_FORMAT, "%s: node %llu: children do not split its rows", path, (unsigned long long)i);
    }
    if (next != nn) return fail(QD_ERR_FORMAT, "%s: %llu nodes are nobody's child", path,
                                (unsigned long long)(nn - next));
    {
        std::vector<uint64_t> seen((n + 63) / 64, 0);
        for (uint64_t i = 0; i < n; i++) {
            const uint32_t r = perm[i];
            if (r >= n || (seen[r / 64] >> (r % 64) & 1)) return fail(QD_ERR_FORMAT, "%s: perm is no permutation", path);
            seen[r / 64] |= 1ull << (r % 64);
        }
    }
    if (abort_requested()) return fail(QD_ERR_ABORTED, "%s: load aborted", path);
    // pass 2: rows and permutation to the device, then everything derived
    hipStream_t s = (hipStream_t)stream;
    qd_tree_s *t = new qd_tree_s();
    t->n = n;
    t->n_nodes = nn;
    t->max_leaf = hd.max_leaf;
    t->has_and = hd.flags & 1u;
    if (hipMalloc((void **)&t->d_sorted, n * 512) != hipSuccess || hipMalloc((void **)&t->d_perm, n * 4) != hipSuccess) {
        tree_release(t);
        return fail(QD_ERR_OOM, "tree allocation failed");
    }
    if (fseek(f, (long)kHeader, SEEK_SET) != 0) {
        tree_release(t);
        return fail(QD_ERR_IO, "%s: seek failed", path);
    }
    uint64_t h2 = kFnvBasis;
    for (uint64_t o = 0; o < n * 512; o += kChunk) {
        const size_t m = (size_t)std::min<uint64_t>(n * 512 - o, kChunk);
        if (!read_hash(f, buf.data(), m, h2, buf) ||
            hipMemcpy(reinterpret_cast<unsigned char *>(t->d_sorted) + o, buf.data(), m, hipMemcpyHostToDevice) !=
                hipSuccess) {
            tree_release(t);
            return fail(QD_ERR_DEVICE, "%s: row upload failed", path);
        }
    }
    if (h2 != h_rows) {
        tree_release(t);
        return fail(QD_ERR_FORMAT, "%s: rows changed while loading", path);
    }
    if (hipMemcpy(t->d_perm, perm.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess) {
        tree_release(t);
        return fail(QD_ERR_DEVICE, "%s: upload failed", path);
    }
    const int rc = tree_finish(t, child, begin, count, (hd.flags & 2u) != 0, s);
    if (rc != QD_OK) return rc;  // tree_finish released t
    *out = t;
    return QD_OK;
}

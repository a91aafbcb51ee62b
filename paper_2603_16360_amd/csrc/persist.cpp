// Index and predictor files: vj_index_save / vj_index_load and
// vj_predictor_save / vj_predictor_load.  The paper builds the merged index
// once and reuses it for any later join and threshold (Section 4.3); these
// files keep it across processes.
//
// Layout (little-endian, this library's own format):
//   8-byte magic, a fixed header of scalars, the arrays back to back, and
//   an FNV-1a 64-bit hash of every preceding byte.  Device arrays are
//   streamed through a host buffer in chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "predictor.h"
#include "vj_internal.h"

namespace vj {
namespace {

constexpr char kIndexMagic[8] = {'V', 'J', 'I', 'D', 'X', '0', '0', '1'};
constexpr char kPredMagic[8] = {'V', 'J', 'M', 'L', 'P', '0', '0', '1'};
constexpr size_t kChunk = (size_t)32 << 20;

struct IndexHeader {
    int64_t nq, nx, repairs;
    int32_t d, dp, R, entry, metric, has_mst, separate, has_nnmap;
};

struct PredHeader {
    int64_t steps;
    int32_t din, h1, h2, k;
};

struct Hash {
    uint64_t h = 1469598103934665603ull;
    void add(const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    }
};

struct Writer {
    FILE *f = nullptr;
    Hash hash;
    std::vector<char> buf;
    explicit Writer(const char *path) : f(std::fopen(path, "wb")) {
        VJ_CHECK(f != nullptr, VJ_ERR_IO, std::string("cannot open for writing: ") + path);
    }
    ~Writer() { if (f) std::fclose(f); }
    void host(const void *p, size_t n) {
        hash.add(p, n);
        VJ_CHECK(std::fwrite(p, 1, n, f) == n, VJ_ERR_IO, "write failed");
    }
    void device(const void *p, size_t n) {
        buf.resize(std::min(n, kChunk));
        for (size_t o = 0; o < n; o += kChunk) {
            const size_t c = std::min(kChunk, n - o);
            VJ_HIP(hipMemcpy(buf.data(), static_cast<const char *>(p) + o, c, hipMemcpyDeviceToHost));
            host(buf.data(), c);
        }
    }
    void close() {
        const uint64_t h = hash.h;
        VJ_CHECK(std::fwrite(&h, 1, 8, f) == 8, VJ_ERR_IO, "write failed");
        VJ_CHECK(std::fclose(f) == 0, VJ_ERR_IO, "close failed");
        f = nullptr;
    }
};

struct Reader {
    FILE *f = nullptr;
    Hash hash;
    std::vector<char> buf;
    explicit Reader(const char *path) : f(std::fopen(path, "rb")) {
        VJ_CHECK(f != nullptr, VJ_ERR_IO, std::string("cannot open for reading: ") + path);
    }
    ~Reader() { if (f) std::fclose(f); }
    void host(void *p, size_t n) {
        VJ_CHECK(std::fread(p, 1, n, f) == n, VJ_ERR_IO, "file is truncated");
        hash.add(p, n);
    }
    void device(void *p, size_t n) {
        buf.resize(std::min(n, kChunk));
        for (size_t o = 0; o < n; o += kChunk) {
            const size_t c = std::min(kChunk, n - o);
            host(buf.data(), c);
            VJ_HIP(hipMemcpy(static_cast<char *>(p) + o, buf.data(), c, hipMemcpyHostToDevice));
        }
    }
    void check_end() {
        const uint64_t want = hash.h;
        uint64_t got = 0;
        VJ_CHECK(std::fread(&got, 1, 8, f) == 8, VJ_ERR_IO, "file is truncated");
        VJ_CHECK(got == want, VJ_ERR_IO, "file checksum mismatch (corrupt file)");
        char extra;
        VJ_CHECK(std::fread(&extra, 1, 1, f) == 0, VJ_ERR_IO, "trailing bytes after the checksum");
    }
};

}  // namespace

void index_save(const Index &ix, const char *path) {
    Writer w(path);
    w.host(kIndexMagic, 8);
    IndexHeader h{ix.nq, ix.nx, ix.repairs, ix.d, ix.dp, ix.R, ix.entry, (int32_t)ix.metric,
                  ix.has_mst ? 1 : 0, ix.separate ? 1 : 0, ix.has_nnmap ? 1 : 0};
    w.host(&h, sizeof(h));
    w.device(ix.vec.p, (size_t)ix.N * ix.dp * sizeof(float));
    w.device(ix.adj.p, (size_t)ix.N * ix.R * sizeof(int32_t));
    w.device(ix.elen.p, (size_t)ix.N * ix.R * sizeof(float));
    if (ix.has_mst && ix.nq > 0) {
        w.device(ix.parent.p, (size_t)ix.nq * sizeof(int32_t));
        w.device(ix.depth.p, (size_t)ix.nq * sizeof(int32_t));
    }
    if (ix.has_nnmap && ix.nq > 0) {
        w.device(ix.nn_w.p, (size_t)ix.nq * sizeof(int32_t));
        w.device(ix.nn_d.p, (size_t)ix.nq * sizeof(double));
        w.device(ix.nn_ood.p, (size_t)ix.nq);
    }
    w.close();
}

void index_load(Index &ix, const char *path, void (*finish)(Index &, hipStream_t), hipStream_t s) {
    Reader r(path);
    char magic[8];
    r.host(magic, 8);
    VJ_CHECK(std::memcmp(magic, kIndexMagic, 8) == 0, VJ_ERR_IO, "not a vj index file");
    IndexHeader h{};
    r.host(&h, sizeof(h));
    VJ_CHECK(h.nq >= 0 && h.nx >= 1 && h.nq + h.nx < ((int64_t)1 << 30) && h.d >= 1 &&
                 h.d <= 1024 && h.dp == padded_dim(h.d) && h.R >= 1 && h.R <= 64 &&
                 h.entry >= 0 && h.entry < h.nq + h.nx && (h.metric == VJ_L2 || h.metric == VJ_IP) &&
                 (h.separate == 0 || h.separate == 1) && (h.has_nnmap == 0 || h.has_nnmap == 1),
             VJ_ERR_IO, "index file header is out of range");
    ix.nq = h.nq; ix.nx = h.nx; ix.N = h.nq + h.nx; ix.d = h.d; ix.dp = h.dp; ix.R = h.R;
    ix.entry = h.entry; ix.metric = (vj_metric)h.metric; ix.repairs = h.repairs;
    ix.separate = h.separate != 0;
    VJ_HIP(hipGetDevice(&ix.device));
    ix.vec.alloc((size_t)ix.N * ix.dp * sizeof(float));
    ix.adj.alloc((size_t)ix.N * ix.R * sizeof(int32_t));
    ix.elen.alloc((size_t)ix.N * ix.R * sizeof(float));
    r.device(ix.vec.p, ix.vec.bytes);
    r.device(ix.adj.p, ix.adj.bytes);
    r.device(ix.elen.p, ix.elen.bytes);
    ix.has_mst = h.has_mst != 0;
    if (ix.has_mst) {
        const size_t nq = (size_t)std::max<int64_t>(ix.nq, 1);
        ix.parent.alloc(nq * sizeof(int32_t));
        ix.depth.alloc(nq * sizeof(int32_t));
        if (ix.nq > 0) {
            r.device(ix.parent.p, (size_t)ix.nq * sizeof(int32_t));
            r.device(ix.depth.p, (size_t)ix.nq * sizeof(int32_t));
        }
    }
    if (h.has_nnmap) {
        const size_t nq = (size_t)std::max<int64_t>(ix.nq, 1);
        ix.nn_w.alloc(nq * sizeof(int32_t));
        ix.nn_d.alloc(nq * sizeof(double));
        ix.nn_ood.alloc(nq);
        if (ix.nq > 0) {
            r.device(ix.nn_w.p, (size_t)ix.nq * sizeof(int32_t));
            r.device(ix.nn_d.p, (size_t)ix.nq * sizeof(double));
            r.device(ix.nn_ood.p, (size_t)ix.nq);
        }
        ix.has_nnmap = true;
    }
    r.check_end();
    finish(ix, s);
}

void predictor_save(const Predictor &p, const char *path) {
    Writer w(path);
    w.host(kPredMagic, 8);
    PredHeader h{p.steps, p.din, p.h1, p.h2, p.k};
    w.host(&h, sizeof(h));
    for (const DevBuf *b : {&p.W1, &p.b1, &p.W2, &p.b2, &p.W3, &p.b3, &p.mu, &p.inv_sigma, &p.m, &p.v})
        w.device(b->p, b->bytes);
    w.close();
}

void predictor_load(Predictor &p, const char *path, hipStream_t s) {
    Reader r(path);
    char magic[8];
    r.host(magic, 8);
    VJ_CHECK(std::memcmp(magic, kPredMagic, 8) == 0, VJ_ERR_IO, "not a vj predictor file");
    PredHeader h{};
    r.host(&h, sizeof(h));
    VJ_CHECK(h.din >= 1 && h.h1 >= 1 && h.h2 >= 1 && h.k >= 1 && h.k <= 64 && h.steps >= 0 &&
                 (int64_t)h.din * h.h1 < ((int64_t)1 << 31) && (int64_t)h.h1 * h.h2 < ((int64_t)1 << 31),
             VJ_ERR_IO, "predictor file header is out of range");
    predictor_init(p, h.din, h.h1, h.h2, h.k, 0, s);
    p.steps = h.steps;
    for (DevBuf *b : {&p.W1, &p.b1, &p.W2, &p.b2, &p.W3, &p.b3, &p.mu, &p.inv_sigma, &p.m, &p.v})
        r.device(b->p, b->bytes);
    r.check_end();
}

}  // namespace vj

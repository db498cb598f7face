// hisq_io.hip -- offline storage of packed fields (the outlook of Sec. 7:
// gauge fields and propagators kept on disk in the bit-packed formats).
// A file is a 128-byte little-endian header followed by the device bytes of
// the packed field(s) verbatim, so a field is written and read back without
// unpacking and keeps the exact bits the kernels read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "hisq_internal.h"

namespace hisq {
namespace {

constexpr char kMagic[8] = {'H', 'I', 'S', 'Q', 'P', 'K', '0', '1'};
constexpr size_t kChunk = size_t(64) << 20;   // staging buffer: 64 MiB of pinned host memory

struct FileHeader {
    char magic[8];
    int32_t kind;          // HISQ_FIELD_SPINOR or HISQ_FIELD_GAUGE
    int32_t fmt;           // spinor or gauge storage format
    int32_t dims[4];       // gauge: lattice extents; spinor: zero
    int64_t nsites;        // spinor: sites; gauge: lattice volume
    int32_t long_recon;    // gauge: long-link storage (18, 12 or 8); spinor: zero
    int32_t reserved0;
    double fat_max, long_max, long_coeff;   // gauge scales (zero for spinors)
    uint64_t bytes0;       // spinor payload, or the fat-link payload
    uint64_t bytes1;       // long-link payload (zero for spinors)
    uint64_t checksum;     // over the payload, see Checksum
    uint8_t reserved1[128 - 96];
};
static_assert(sizeof(FileHeader) == 128, "header layout");

// FNV-1a over little-endian 64-bit words (a short tail padded with zeros)
struct Checksum {
    uint64_t h = 0xcbf29ce484222325ull;
    void add(const unsigned char *p, size_t n) {
        size_t i = 0;
        for (; i + 8 <= n; i += 8) {
            uint64_t w;
            std::memcpy(&w, p + i, 8);
            h = (h ^ w) * 0x100000001b3ull;
        }
        if (i < n) {
            uint64_t w = 0;
            std::memcpy(&w, p + i, n - i);
            h = (h ^ w) * 0x100000001b3ull;
        }
    }
};

struct File {
    FILE *f = nullptr;
    File(const char *path, const char *mode) : f(std::fopen(path, mode)) {}
    ~File() {
        if (f) std::fclose(f);
    }
};

struct Pinned {
    void *p = nullptr;
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
};

// device -> file through the pinned staging buffer.  The checksum runs over
// each payload in the same kChunk pieces (a multiple of 8 bytes) on both
// sides, so writer and reader sum the same words.
hisq_status write_payload(FILE *f, const void *src, size_t n, Checksum &ck, hipStream_t st, void *stage) {
    const char *s = static_cast<const char *>(src);
    for (size_t off = 0; off < n; off += kChunk) {
        const size_t m = std::min(kChunk, n - off);
        HISQ_TRY_HIP(hipMemcpyAsync(stage, s + off, m, hipMemcpyDeviceToHost, st));
        HISQ_TRY_HIP(hipStreamSynchronize(st));
        ck.add(static_cast<const unsigned char *>(stage), m);
        if (std::fwrite(stage, 1, m, f) != m) return set_error(HISQ_EIO, "write failed");
    }
    return HISQ_OK;
}

hisq_status read_payload(FILE *f, void *dst, size_t n, Checksum &ck, hipStream_t st, void *stage) {
    char *d = static_cast<char *>(dst);
    for (size_t off = 0; off < n; off += kChunk) {
        const size_t m = std::min(kChunk, n - off);
        if (std::fread(stage, 1, m, f) != m) return set_error(HISQ_EIO, "file shorter than its header states");
        ck.add(static_cast<const unsigned char *>(stage), m);
        HISQ_TRY_HIP(hipMemcpyAsync(d + off, stage, m, hipMemcpyHostToDevice, st));
        HISQ_TRY_HIP(hipStreamSynchronize(st));
    }
    return HISQ_OK;
}

hisq_status read_header(FILE *f, FileHeader &h) {
    if (std::fread(&h, 1, sizeof(h), f) != sizeof(h)) return set_error(HISQ_EIO, "file shorter than a header");
    if (std::memcmp(h.magic, kMagic, 8) != 0) return set_error(HISQ_EIO, "not a packed-field file");
    if (h.kind == HISQ_FIELD_SPINOR) {
        if (h.fmt < 0 || h.fmt > HISQ_SPINOR_INT24 || h.nsites < 0 ||
            h.bytes0 != spinor_field_bytes((size_t)h.nsites, h.fmt) || h.bytes1 != 0)
            return set_error(HISQ_EIO, "inconsistent spinor header");
    } else if (h.kind == HISQ_FIELD_GAUGE) {
        if (h.fmt < 0 || h.fmt > HISQ_GAUGE_SX24 || !dims_ok(h.dims) ||
            (h.long_recon != HISQ_RECON_18 && h.long_recon != HISQ_RECON_12 && h.long_recon != HISQ_RECON_8))
            return set_error(HISQ_EIO, "inconsistent gauge header");
        if (h.bytes0 != hisq_gauge_bytes(h.dims, h.fmt) ||
            h.bytes1 != hisq_gauge_long_bytes(h.dims, h.fmt, h.long_recon))
            return set_error(HISQ_EIO, "gauge header sizes do not match its format");
    } else {
        return set_error(HISQ_EIO, "unknown field kind %d", h.kind);
    }
    return HISQ_OK;
}

// the payload ends exactly where the header says
hisq_status check_end(FILE *f, const Checksum &ck, const FileHeader &h) {
    if (std::fgetc(f) != EOF) return set_error(HISQ_EIO, "file longer than its header states");
    if (ck.h != h.checksum) return set_error(HISQ_EIO, "checksum mismatch (the destination holds the file's bytes)");
    return HISQ_OK;
}

}  // namespace
}  // namespace hisq

using namespace hisq;

extern "C" hisq_status hisq_field_info(const char *path, hisq_field_header *info) {
    if (!path || !info) return set_error(HISQ_EINVAL, "hisq_field_info: null pointer");
    File f(path, "rb");
    if (!f.f) return set_error(HISQ_EIO, "hisq_field_info: cannot open %s", path);
    FileHeader h;
    HISQ_TRY(read_header(f.f, h));
    info->kind = h.kind;
    info->fmt = h.fmt;
    for (int k = 0; k < 4; k++) info->dims[k] = h.dims[k];
    info->nsites = (long)h.nsites;
    info->long_recon = h.long_recon;
    info->bytes0 = (size_t)h.bytes0;
    info->bytes1 = (size_t)h.bytes1;
    return HISQ_OK;
}

extern "C" hisq_status hisq_spinor_save(const char *path, const void *src, long nsites, int spinor_fmt, void *stream) {
    if (!path || !src) return set_error(HISQ_EINVAL, "hisq_spinor_save: null pointer");
    if (nsites < 0 || spinor_fmt < 0 || spinor_fmt > HISQ_SPINOR_INT24)
        return set_error(HISQ_EINVAL, "hisq_spinor_save: bad size or format");
    FileHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kMagic, 8);
    h.kind = HISQ_FIELD_SPINOR;
    h.fmt = spinor_fmt;
    h.nsites = nsites;
    h.bytes0 = spinor_field_bytes((size_t)nsites, spinor_fmt);
    File f(path, "wb");
    if (!f.f) return set_error(HISQ_EIO, "hisq_spinor_save: cannot create %s", path);
    Pinned stage;
    HISQ_TRY_HIP(hipHostMalloc(&stage.p, kChunk, hipHostMallocDefault));
    Checksum ck;
    // header first with a zero checksum, rewritten once the payload is summed
    if (std::fwrite(&h, 1, sizeof(h), f.f) != sizeof(h)) return set_error(HISQ_EIO, "hisq_spinor_save: write failed");
    HISQ_TRY(write_payload(f.f, src, (size_t)h.bytes0, ck, (hipStream_t)stream, stage.p));
    h.checksum = ck.h;
    if (std::fseek(f.f, 0, SEEK_SET) != 0 || std::fwrite(&h, 1, sizeof(h), f.f) != sizeof(h) || std::fflush(f.f) != 0)
        return set_error(HISQ_EIO, "hisq_spinor_save: write failed");
    return HISQ_OK;
}

extern "C" hisq_status hisq_spinor_load(const char *path, void *dst, long nsites, int spinor_fmt, void *stream) {
    if (!path || !dst) return set_error(HISQ_EINVAL, "hisq_spinor_load: null pointer");
    File f(path, "rb");
    if (!f.f) return set_error(HISQ_EIO, "hisq_spinor_load: cannot open %s", path);
    FileHeader h;
    HISQ_TRY(read_header(f.f, h));
    if (h.kind != HISQ_FIELD_SPINOR || h.fmt != spinor_fmt || h.nsites != nsites)
        return set_error(HISQ_EINVAL, "hisq_spinor_load: the file holds kind %d format %d with %lld sites", h.kind,
                         h.fmt, (long long)h.nsites);
    Pinned stage;
    HISQ_TRY_HIP(hipHostMalloc(&stage.p, kChunk, hipHostMallocDefault));
    Checksum ck;
    HISQ_TRY(read_payload(f.f, dst, (size_t)h.bytes0, ck, (hipStream_t)stream, stage.p));
    return check_end(f.f, ck, h);
}

extern "C" hisq_status hisq_gauge_save(const char *path, const hisq_gauge *g, void *stream) {
    if (!path || !g || !g->fat || !g->lng) return set_error(HISQ_EINVAL, "hisq_gauge_save: null pointer");
    if (!dims_ok(g->dims) || g->fmt < 0 || g->fmt > HISQ_GAUGE_SX24 ||
        (g->long_recon != HISQ_RECON_18 && g->long_recon != HISQ_RECON_12 && g->long_recon != HISQ_RECON_8))
        return set_error(HISQ_EINVAL, "hisq_gauge_save: descriptor not filled by hisq_gauge_pack");
    FileHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kMagic, 8);
    h.kind = HISQ_FIELD_GAUGE;
    h.fmt = g->fmt;
    for (int k = 0; k < 4; k++) h.dims[k] = g->dims[k];
    h.nsites = (int64_t)g->dims[0] * g->dims[1] * g->dims[2] * g->dims[3];
    h.long_recon = g->long_recon;
    h.fat_max = g->fat_max;
    h.long_max = g->long_max;
    h.long_coeff = g->long_coeff;
    h.bytes0 = hisq_gauge_bytes(g->dims, g->fmt);
    h.bytes1 = hisq_gauge_long_bytes(g->dims, g->fmt, g->long_recon);
    File f(path, "wb");
    if (!f.f) return set_error(HISQ_EIO, "hisq_gauge_save: cannot create %s", path);
    Pinned stage;
    HISQ_TRY_HIP(hipHostMalloc(&stage.p, kChunk, hipHostMallocDefault));
    Checksum ck;
    if (std::fwrite(&h, 1, sizeof(h), f.f) != sizeof(h)) return set_error(HISQ_EIO, "hisq_gauge_save: write failed");
    HISQ_TRY(write_payload(f.f, g->fat, (size_t)h.bytes0, ck, (hipStream_t)stream, stage.p));
    HISQ_TRY(write_payload(f.f, g->lng, (size_t)h.bytes1, ck, (hipStream_t)stream, stage.p));
    h.checksum = ck.h;
    if (std::fseek(f.f, 0, SEEK_SET) != 0 || std::fwrite(&h, 1, sizeof(h), f.f) != sizeof(h) || std::fflush(f.f) != 0)
        return set_error(HISQ_EIO, "hisq_gauge_save: write failed");
    return HISQ_OK;
}

extern "C" hisq_status hisq_gauge_load(const char *path, hisq_gauge *g, void *fat_dst, size_t fat_bytes,
                                       void *long_dst, size_t long_bytes, void *stream) {
    if (!path || !g || !fat_dst || !long_dst) return set_error(HISQ_EINVAL, "hisq_gauge_load: null pointer");
    if (!aligned16(fat_dst) || !aligned16(long_dst)) return set_error(HISQ_EALIGN, "hisq_gauge_load: unaligned pointer");
    File f(path, "rb");
    if (!f.f) return set_error(HISQ_EIO, "hisq_gauge_load: cannot open %s", path);
    FileHeader h;
    HISQ_TRY(read_header(f.f, h));
    if (h.kind != HISQ_FIELD_GAUGE) return set_error(HISQ_EINVAL, "hisq_gauge_load: the file holds a spinor field");
    if (fat_bytes < h.bytes0 || long_bytes < h.bytes1)
        return set_error(HISQ_EINVAL, "hisq_gauge_load: buffers of %zu and %zu bytes, need %llu and %llu", fat_bytes,
                         long_bytes, (unsigned long long)h.bytes0, (unsigned long long)h.bytes1);
    Pinned stage;
    HISQ_TRY_HIP(hipHostMalloc(&stage.p, kChunk, hipHostMallocDefault));
    Checksum ck;
    HISQ_TRY(read_payload(f.f, fat_dst, (size_t)h.bytes0, ck, (hipStream_t)stream, stage.p));
    HISQ_TRY(read_payload(f.f, long_dst, (size_t)h.bytes1, ck, (hipStream_t)stream, stage.p));
    HISQ_TRY(check_end(f.f, ck, h));
    for (int k = 0; k < 4; k++) g->dims[k] = h.dims[k];
    g->fmt = h.fmt;
    g->fat = fat_dst;
    g->lng = long_dst;
    g->fat_max = h.fat_max;
    g->long_max = h.long_max;
    g->long_recon = h.long_recon;
    g->long_coeff = h.long_coeff;
    return HISQ_OK;
}

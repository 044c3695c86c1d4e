// autotune.hip -- host side of the kernel-choice tuner (gsyeig_autotune):
// the JSON cache of tuned choices keyed by (architecture, precision,
// n-bucket) and the synthetic operands the measurements run on.
//
// Cache format (written and read only by this file):
//   {"arch": "gfx950:...", "entries": [
//     {"prec": 0, "n_bucket": 16384, "trsv_block": 512, "trsv_sweep": 0,
//      "gemm_big_min": 2048, "op_ms": 0.76, "gemm_ms": 1.92}, ...]}
// Entries of other architectures are kept when the file is rewritten.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "internal.h"

namespace {

// SplitMix64 finaliser as a hash of (seed, i, j) -> uniform [0, 1)
__device__ __forceinline__ double hash01(uint64_t seed, int64_t i, int64_t j)
{
    uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull + (uint64_t)j * 0xD1B54A32D192ED03ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

// U: upper triangular, diagonal in [1, 2], strict upper in [-1, 1] / sqrt(n);
// A: symmetric with entries in [-1, 1].  Row-major, leading dimension ld.
__global__ void k_synth(double *U, double *A, int64_t ld, int64_t n, uint64_t seed)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= n || i >= n) return;
    double u = 0.0;
    if (j == i) u = 1.0 + hash01(seed, i, j);
    else if (j > i) u = (2.0 * hash01(seed, i, j) - 1.0) / sqrt((double)n);
    U[i * ld + j] = u;
    const int64_t a = i < j ? i : j, b = i < j ? j : i;
    A[i * ld + j] = 2.0 * hash01(seed ^ 0x5DEECE66Dull, a, b) - 1.0;
}

const char *skip_ws(const char *p)
{
    while (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r' || *p == ',') ++p;
    return p;
}

// value of "key": number inside the object text [b, e)
bool num_field(const char *b, const char *e, const char *key, double *v)
{
    std::string k = std::string("\"") + key + "\"";
    const char *p = strstr(b, k.c_str());
    if (!p || p >= e) return false;
    p = strchr(p + k.size(), ':');
    if (!p || p >= e) return false;
    *v = strtod(p + 1, nullptr);
    return true;
}

}  // namespace

int launch_synth_operands(double *U, double *A, int64_t ld, int64_t n, uint64_t seed, hipStream_t st)
{
    for (int64_t r0 = 0; r0 < n; r0 += 65535) {
        const int64_t nr = (n - r0 < 65535) ? n - r0 : 65535;
        hipLaunchKernelGGL(k_synth, dim3((unsigned)cdiv(n, 256), (unsigned)nr), dim3(256), 0, st, U + r0 * ld,
                           A + r0 * ld, ld, n, seed);
        if (hipGetLastError() != hipSuccess) return GSYEIG_EHIP;
    }
    return 0;
}

// Reads the entries of `arch` from the cache file (missing file: none);
// *others receives the text of other architectures' entries verbatim.
int tune_cache_load(const char *path, const char *arch, std::vector<TuneEntry> *out, std::string *others)
{
    out->clear();
    others->clear();
    FILE *f = fopen(path, "rb");
    if (!f) return 0;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    fclose(f);
    // one object per architecture: {"arch": "...", "entries": [ {...}, ... ]}
    const char *p = text.c_str();
    while ((p = strstr(p, "\"arch\"")) != nullptr) {
        const char *q = strchr(p, ':');
        if (!q) break;
        q = strchr(q, '"');
        if (!q) break;
        const char *qe = strchr(q + 1, '"');
        if (!qe) break;
        const std::string a(q + 1, qe);
        const char *lb = strchr(qe, '[');
        if (!lb) break;
        const char *rb = strchr(lb, ']');
        if (!rb) break;
        if (a == arch) {
            const char *o = lb + 1;
            while (true) {
                o = skip_ws(o);
                if (*o != '{') break;
                const char *oe = strchr(o, '}');
                if (!oe || oe > rb) break;
                TuneEntry t{};
                double v;
                if (num_field(o, oe, "prec", &v)) t.prec = (int)v;
                if (num_field(o, oe, "n_bucket", &v)) t.n_bucket = (int64_t)v;
                if (num_field(o, oe, "trsv_block", &v)) t.trsv_block = (int)v;
                if (num_field(o, oe, "trsv_sweep", &v)) t.trsv_sweep = (int)v;
                if (num_field(o, oe, "gemm_big_min", &v)) t.gemm_big_min = (int64_t)v;
                if (num_field(o, oe, "op_ms", &v)) t.op_ms = v;
                if (num_field(o, oe, "gemm_ms", &v)) t.gemm_ms = v;
                if (t.n_bucket > 0 && (t.trsv_block == 64 || t.trsv_block == 512)) out->push_back(t);
                o = oe + 1;
            }
        } else {
            const char *ob = p;  // back to this architecture's '{'
            while (ob > text.c_str() && *ob != '{') --ob;
            const char *oe = strchr(rb, '}');
            if (oe) {
                if (!others->empty()) *others += ",\n";
                others->append(ob, oe + 1);
            }
        }
        p = rb;
    }
    return 0;
}

int tune_cache_store(const char *path, const char *arch, const std::vector<TuneEntry> &entries,
                     const std::string &others)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return GSYEIG_EHIP;
    fprintf(f, "[\n");
    if (!others.empty()) fprintf(f, "%s,\n", others.c_str());
    fprintf(f, "{\"arch\": \"%s\", \"entries\": [\n", arch);
    for (size_t k = 0; k < entries.size(); ++k) {
        const TuneEntry &t = entries[k];
        fprintf(f,
                "  {\"prec\": %d, \"n_bucket\": %lld, \"trsv_block\": %d, \"trsv_sweep\": %d, \"gemm_big_min\": %lld, "
                "\"op_ms\": %.6f, \"gemm_ms\": %.6f}%s\n",
                t.prec, (long long)t.n_bucket, t.trsv_block, t.trsv_sweep, (long long)t.gemm_big_min, t.op_ms,
                t.gemm_ms, k + 1 < entries.size() ? "," : "");
    }
    fprintf(f, "]}\n]\n");
    if (fclose(f) != 0) return GSYEIG_EHIP;
    return rename(tmp.c_str(), path) == 0 ? 0 : GSYEIG_EHIP;
}

// Internal declarations shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/onng.h"

namespace onng {

// ---------------------------------------------------------------- errors --

// Thread-local error message behind onng_last_error().
void set_error(const std::string &msg);
const char *get_error();

#define ONNG_CHECK_ARG(cond, msg)                                     \
    do {                                                              \
        if (!(cond)) {                                                \
            ::onng::set_error(std::string(__func__) + ": " + (msg));  \
            return ONNG_ERR_INVALID_ARG;                              \
        }                                                             \
    } while (0)

#define ONNG_HIP(call)                                                            \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::onng::set_error(std::string(__func__) + ": " #call ": " +          \
                              hipGetErrorString(e_));                             \
            return ONNG_ERR_DEVICE;                                               \
        }                                                                         \
    } while (0)

// ------------------------------------------------------------- dtypes ----

// smallest pitch of FP8 rows that keep their scale in the last 4 bytes,
// past every 16-byte piece that holds components
inline int64_t fp8_inrow_pitch(int32_t dim) { return ((int64_t)dim + 15) / 16 * 16 + 16; }

inline int elem_bytes(int dtype) {
    switch (dtype) {
    case ONNG_U8: return 1;
    case ONNG_F32: return 4;
    case ONNG_F16: return 2;
    case ONNG_BF16: return 2;
    case ONNG_FP8_E4M3: return 1;
    }
    return 0;
}

// u8 + L2SQ: exact int32 distances; everything else f32.
inline bool int_dist(int dtype, int metric) { return dtype == ONNG_U8 && metric == ONNG_L2SQ; }

onng_status check_vectors(const onng_vectors *v, const char *what);

// Carve aligned sub-buffers out of a caller workspace.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *p) : base(static_cast<char *>(p)) {}
    template <typename T>
    T *take(size_t count, size_t align = 256) {
        off = (off + align - 1) / align * align;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t size() const { return off; }
};

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

int device_cu_count();

// ------------------------------------------------------ device helpers ---

// Monotone map of a float to uint32 (total order of the values).
__device__ __host__ inline uint32_t ord_f32(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __host__ inline float unord_f32(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}

// Sort key of (distance, id): distance in the high word (int distances are
// < 2^24 and used as is), id in the low word.
__device__ __host__ inline uint64_t make_key(uint32_t dord, uint32_t id) {
    return (uint64_t(dord) << 32) | id;
}
constexpr uint64_t KEY_MAX = ~uint64_t(0);

// ------------------------------------------------------------ launches ---

// Top-k of distances (the k-NN graph, seeds, ground truth).
onng_status launch_topk(const onng_vectors *Q, const onng_vectors *B, const int32_t *cand,
                        int64_t n_cand, int32_t k, int32_t exclude_self, int32_t *ids,
                        void *dists, void *ws, size_t ws_bytes, hipStream_t st);
size_t topk_ws_size(const onng_vectors *Q, const onng_vectors *B, int64_t n_cand, int32_t k);

}  // namespace onng

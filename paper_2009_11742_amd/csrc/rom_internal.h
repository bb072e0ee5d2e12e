// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rom.h"

namespace rom {

// Row tile of the rank-2 MFMA kernel: one v_mfma_f32_4x4x1f32 (16 blocks)
// covers 64 operator rows x 4 sample columns for one k.
constexpr int kTileRows = 64;
// Sample columns owned by one workgroup of the rank-2 FP32 kernel.
constexpr int kColBlock = 4;
// Largest Kv_pad + Ks_pad the LDS-resident state of the rank-2 kernels holds.
constexpr int kMaxPadSum = 4096;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace rom

struct rom_ctx {
    int device = 0;
    int kv = 0, ks = 0;        // reduced sizes
    int kvp = 0, ksp = 0;      // padded to multiples of 64
    double dt = 0.0;           // as given
    rom_dtype op_type = ROM_F64, state_type = ROM_F64;
    uint32_t flags = 0;
    bool skew = false;         // Asv == -Avs^T exactly

    // Column-major operators in the state type (rank-1 GEMV and FP64 path):
    // Avs kv x ks (ld kv), Asv ks x kv (ld ks).
    void *avs_cm = nullptr, *asv_cm = nullptr;
    // FP32 operators packed for the 4x4x1 MFMA kernel:
    // avs_pk[t][k/4][lane][k%4] = Avs[64 t + lane][k], zero padded to kvp x ksp;
    // asv_pk likewise for Asv (ksp x kvp).
    float *avs_pk = nullptr, *asv_pk = nullptr;
    // Source vector in the state type, zero padded to kvp entries.
    void *b = nullptr;
    // Transposed operators (column-major, state type) for the adjoint, lazily.
    void *avs_t = nullptr, *asv_t = nullptr;
    // Device status word (in-kernel errors).
    int *status = nullptr;
};

namespace rom {

struct Rank2Args {
    const void *avs;      // packed (F32 MFMA) or column-major (VALU path)
    const void *asv;
    const void *b;        // kvp entries
    const void *c;        // kv entries or null
    const double *mu;     // M
    void *V, *S;          // caller states (column-major, ld kv / ks)
    double *J;            // M or null (accumulated)
    double *y;            // nsteps x M or null
    int kv, ks, kvp, ksp, M;
    int64_t n0, nsteps;
    double dt;            // FP64 step (forcing time t_n = n * dt)
};

// Launchers (return hipSuccess or the launch error).
hipError_t launch_rank2_f32_mfma(const Rank2Args &a, hipStream_t st);
template <typename T>
hipError_t launch_rank2_valu(const Rank2Args &a, hipStream_t st);

template <typename T>
hipError_t launch_rank1_step(const void *avs_cm, const void *asv_cm, const void *b, int kv,
                             int ks, double dt, int64_t n, double mu, void *v, void *s,
                             hipStream_t st);

// Setup kernels: FP64 staging -> state-type column-major copies and packed
// MFMA panels.
hipError_t launch_convert(const double *src, void *dst, int64_t n, rom_dtype to, hipStream_t st);
hipError_t launch_pack_f32(const double *A, int rows, int cols, int rowsp, int colsp, float *pk,
                           hipStream_t st);

}  // namespace rom

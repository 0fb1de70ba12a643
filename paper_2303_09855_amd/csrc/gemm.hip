// FP32 GEMM on the CDNA4 matrix cores: C[M][N] = A[M][K] * B[N][K]^T.
//
// Used for the random rotation y = P x of Section 3.1 (X * P^T for a batch of
// rows; queries in the query phase, base vectors and centres in the index
// phase) and for the query-centre inner products of IVF probe selection.
//
// Tiling: a (2WT)x(2WT) output tile per 256-thread workgroup, 2x2 waves of
// WT x WT, each wave a (WT/16)x(WT/16) grid of v_mfma_f32_16x16x4_f32 tiles.
// WT = 64 (128x128 tiles, 64 accumulators per lane) by default; WT = 32
// (64x64 tiles) when the 128-tile grid would leave most CUs idle (e.g. the
// rotation of a batch of 1,000 queries).  K is staged through LDS 16 at a
// time in k-major order so that each MFMA operand fetch is 16 consecutive
// floats.  Rows and columns past M / N are zero-filled on load and masked
// on store; K must be a multiple of 4.
#include "common.h"

namespace ads {

namespace {

constexpr int BK = 16, PADL = 4;

typedef float v4f __attribute__((ext_vector_type(4)));

template <int WT>
__global__ __launch_bounds__(ADS_WG) void gemm_nt_f32_kernel(
    const float *__restrict__ A, int64_t lda, const float *__restrict__ B, int64_t ldb,
    float *__restrict__ C, int64_t ldc, int64_t M, int64_t N, int K) {
    constexpr int BM = 2 * WT, BN = 2 * WT, TT = WT / 16;
    __shared__ float As[BK][BM + PADL];
    __shared__ float Bs[BK][BN + PADL];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;

    v4f acc[TT][TT];
#pragma unroll
    for (int i = 0; i < TT; ++i)
#pragma unroll
        for (int j = 0; j < TT; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += BK) {
        // BM rows x 16 k = BM * 4 float4 per operand, BM / 64 per thread.
#pragma unroll
        for (int t = 0; t < BM / 64; ++t) {
            int idx = tid + t * ADS_WG;
            int row = idx >> 2, kq = (idx & 3) * 4;
            int kk = k0 + kq;
            float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
            if (m0 + row < M && kk < K) va = *reinterpret_cast<const float4 *>(A + (m0 + row) * lda + kk);
            if (n0 + row < N && kk < K) vb = *reinterpret_cast<const float4 *>(B + (n0 + row) * ldb + kk);
            As[kq + 0][row] = va.x; As[kq + 1][row] = va.y; As[kq + 2][row] = va.z; As[kq + 3][row] = va.w;
            Bs[kq + 0][row] = vb.x; Bs[kq + 1][row] = vb.y; Bs[kq + 2][row] = vb.z; Bs[kq + 3][row] = vb.w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float a[TT], b[TT];
            const int kr = kk + (lane >> 4), c = lane & 15;
#pragma unroll
            for (int i = 0; i < TT; ++i) a[i] = As[kr][wm * WT + i * 16 + c];
#pragma unroll
            for (int j = 0; j < TT; ++j) b[j] = Bs[kr][wn * WT + j * 16 + c];
#pragma unroll
            for (int i = 0; i < TT; ++i)
#pragma unroll
                for (int j = 0; j < TT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // D[4*(lane/16) + r][lane % 16] of each 16x16 tile sits in acc[.][.][r].
    const int cc = lane & 15, rb = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < TT; ++i)
#pragma unroll
        for (int j = 0; j < TT; ++j) {
            int64_t col = n0 + wn * WT + j * 16 + cc;
            if (col >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int64_t row = m0 + wm * WT + i * 16 + rb + r;
                if (row < M) C[row * ldc + col] = acc[i][j][r];
            }
        }
}

template <int WT>
void gemm_launch(const float *A, int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc, int64_t M,
                 int64_t N, int K, hipStream_t s) {
    constexpr int BM = 2 * WT, BN = 2 * WT;
    const int64_t gx = (N + BN - 1) / BN;
    // grid.y is limited to 65535: split tall problems into row slabs.
    const int64_t max_rows = (int64_t)65535 * BM;
    for (int64_t r0 = 0; r0 < M; r0 += max_rows) {
        int64_t rows = M - r0 < max_rows ? M - r0 : max_rows;
        dim3 grid((unsigned)gx, (unsigned)((rows + BM - 1) / BM));
        hipLaunchKernelGGL(gemm_nt_f32_kernel<WT>, grid, dim3(ADS_WG), 0, s, A + r0 * lda, lda, B, ldb,
                           C + r0 * ldc, ldc, rows, N, K);
    }
}

}  // namespace

hipError_t gemm_nt_f32(const float *A, int64_t lda, const float *B, int64_t ldb, float *C,
                       int64_t ldc, int64_t M, int64_t N, int K, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t tiles128 = ((M + 127) / 128) * ((N + 127) / 128);
    // 64x64 tiles until there are enough 128x128 tiles for four per CU
    if (tiles128 < 1024)
        gemm_launch<32>(A, lda, B, ldb, C, ldc, M, N, K, s);
    else
        gemm_launch<64>(A, lda, B, ldb, C, ldc, M, N, K, s);
    return hipGetLastError();
}

}  // namespace ads

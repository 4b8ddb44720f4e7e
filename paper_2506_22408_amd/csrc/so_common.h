// so_common.h -- device helpers shared by the shadow-overlap kernels:
// complex arithmetic on double2, 64-lane shuffles, DPP row broadcasts and
// reductions, and the node table passed to the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>
#include <utility>

// complex helpers on double2 (x = re, y = im)
__device__ __forceinline__ double2 c_make(double r, double i) { double2 v; v.x = r; v.y = i; return v; }
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return c_make(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return c_make(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_neg(double2 a) { return c_make(-a.x, -a.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return c_make(a.x * s, a.y * s); }
__device__ __forceinline__ double2 c_conj(double2 a) { return c_make(a.x, -a.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
    return c_make(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// c + a * b
__device__ __forceinline__ double2 c_fma(double2 a, double2 b, double2 c) {
    return c_make(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double c_abs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ double2 c_sel(bool p, double2 a, double2 b) { return c_make(p ? a.x : b.x, p ? a.y : b.y); }
// principal complex logarithm, log|a| + i Arg a with Arg in (-pi, pi]
__device__ __forceinline__ double2 c_log(double2 a) { return c_make(log(hypot(a.x, a.y)), atan2(a.y, a.x)); }
// 1/a for a != 0 (scaled to avoid overflow of |a|^2)
__device__ __forceinline__ double2 c_inv(double2 a) {
    const double s = fmax(fabs(a.x), fabs(a.y));
    const double2 b = c_scale(a, 1.0 / s);
    return c_scale(c_conj(b), 1.0 / (s * c_abs2(b)));
}

// sums and broadcasts over groups of W lanes (ds_bpermute based)
template <int W>
__device__ __forceinline__ double grp_sum(double v) {
#pragma unroll
    for (int off = W / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
}
template <int W>
__device__ __forceinline__ double2 grp_bcast(double2 v, int src) {
    return c_make(__shfl(v.x, src, W), __shfl(v.y, src, W));
}

// ---- DPP within 16-lane rows ------------------------------------------------
// Every move below writes every lane (all row and bank masks set, and each
// pattern reads a lane of the same row), so no lane keeps its old value: the
// moves take no "old" operand and the compiler need not copy the source into
// the destination first.
// a 32-bit DPP move applied to both halves of a double
template <int CTRL>
__device__ __forceinline__ double dpp_f64_32(double v) {
    const long long b = __double_as_longlong(v);
    int lo = (int)b, hi = (int)(b >> 32);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
// broadcast lane SRC of each 16-lane row to the whole row (row_newbcast, a
// 64-bit DPP move)
template <int SRC>
__device__ __forceinline__ double bc16(double v) {
    long long b = __double_as_longlong(v);
    b = __builtin_amdgcn_mov_dpp(b, 0x150 + SRC, 0xf, 0xf, false);
    return __longlong_as_double(b);
}
template <int SRC>
__device__ __forceinline__ double2 bc16c(double2 v) { return c_make(bc16<SRC>(v.x), bc16<SRC>(v.y)); }
// the same broadcast with an artificial data dependence on `dep` (an empty
// asm, no instruction): it cannot be scheduled before `dep` exists, which
// bounds how far the scheduler hoists broadcasts ahead of their use
template <int SRC>
__device__ __forceinline__ double bc16d(double v, double dep) {
    asm("" : "+v"(v) : "v"(dep));
    return bc16<SRC>(v);
}
template <int SRC>
__device__ __forceinline__ double2 bc16cd(double2 v, double dep) {
    return c_make(bc16d<SRC>(v.x, dep), bc16d<SRC>(v.y, dep));
}
// sum over the 16 lanes of a row (rotations: every lane gets the total)
__device__ __forceinline__ double sum16(double v) {
    v += dpp_f64_32<0x128>(v);   // row_ror:8
    v += dpp_f64_32<0x124>(v);   // row_ror:4
    v += dpp_f64_32<0x122>(v);   // row_ror:2
    v += dpp_f64_32<0x121>(v);   // row_ror:1
    return v;
}
// lane 15-i of the row (row_mirror) and lane 7-i of each half row (row_half_mirror)
// 1/x for finite x != 0: the hardware reciprocal refined by two Newton steps
// (each squares the relative error), so the result is within an ulp or two.
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
// 1/a for a != 0, scaled so that |a|^2 cannot overflow or underflow
__device__ __forceinline__ double2 c_inv_nr(double2 a) {
    const double rs = rcp_nr(fmax(fabs(a.x), fabs(a.y)));
    const double2 b = c_scale(a, rs);          // largest component +-1
    return c_scale(c_conj(b), rcp_nr(c_abs2(b)) * rs);
}

// wave-wide maximum of unsigned keys, returned uniformly: DPP within each
// 16-lane row (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror leave every lane of a row with the row's maximum), then the four
// rows on the scalar unit
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
    v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xf, 0xf, false));
    const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
    const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
    const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
    const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
    return max(max(a, b), max(c, d));
}

__device__ __forceinline__ double2 mirror16c(double2 v) { return c_make(dpp_f64_32<0x140>(v.x), dpp_f64_32<0x140>(v.y)); }
__device__ __forceinline__ double2 mirror8c(double2 v) { return c_make(dpp_f64_32<0x141>(v.x), dpp_f64_32<0x141>(v.y)); }

// 64-bit counter type of device atomics (the full-size queue)
typedef unsigned long long so_u64;

// ---- pairs left for the full-size path -----------------------------------------
// A pair that the elimination flags is queued for the full-size path; when
// the queue is full its slot in the pair array receives this quiet-NaN bit
// pattern instead (both halves), and the full-size kernel finds it there by a
// scan.  No arithmetic result has this payload.
#define SO_PAIR_MARK 0x7ff85a5e0fa11bacll
__device__ __forceinline__ double2 so_pair_mark() {
    const double v = __longlong_as_double(SO_PAIR_MARK);
    return c_make(v, v);
}
__device__ __forceinline__ bool so_is_pair_mark(double2 v) {
    return __double_as_longlong(v.x) == SO_PAIR_MARK && __double_as_longlong(v.y) == SO_PAIR_MARK;
}

// ---- node table ---------------------------------------------------------------
// Node matrices are B + c J in the row order [occupied, empty] (see
// so_prep.h).  Q(c) = Pf(B + c J) is a polynomial of degree ne = n - eta in c
// (J has rank 2 ne), and the estimator is a fixed linear functional of its
// coefficients, whatever nodes the caller names.  The kernels therefore
// evaluate Q at ne + 1 points e_j of the unit circle (the roots of unity
// turned by a third of a step) and weigh the values by v_j,
// which carry the interpolation, the inverse-channel factors, the
// estimator's prefactor and the sign of the row permutation.
#define SO_KMAX 49
struct NodeTab {
    double2 e[SO_KMAX];
    double2 v[SO_KMAX];
    int K;    // the caller's node count (validated; the estimator does not depend on it)
    int Ke;   // ne + 1
};
// the reduced-path part of the table, for kernels that need nothing else
struct RedTab {
    double2 e[SO_KMAX];
    double2 v[SO_KMAX];
};

#define SO_NMAX 32
#define SO_NMAX_SUPPORTED 24
#define SO_MMAX 48

// ---- MFMA operand order of the d x d walker and shadow matrices --------------
// v_mfma_f64_16x16x4f64 reads, in lane l at k-step kk of row tile I, the A
// element M[16 I + l%16][4 kk + l/16] (and the B element B[4 kk + l/16][16 J +
// l%16]); register r of its 16 x 16 accumulator holds D[4 r + l/16][l%16].
// The walker matrices Xall and the shadow covariances C' are stored padded
// with zeros to DP = 16 T (T = ceil(2n/16)) in that A order, two k-steps per
// lane as one double2, so that a wave fetches one operand pair with a single
// coalesced 1 KiB access:
//   flat(I, kk, l) = ((I (KK/2) + kk/2) 64 + l) 2 + kk % 2,  KK = 4 T.
typedef double so_d4 __attribute__((ext_vector_type(4)));
typedef float so_f4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline int so_tiles(int n) { return (2 * n + 15) / 16; }

__device__ __forceinline__ int ao_index(int row, int col, int T) {
    const int I = row >> 4, kk = col >> 2, l = (row & 15) | ((col & 3) << 4);
    return ((I * 2 * T + (kk >> 1)) * 64 + l) * 2 + (kk & 1);
}
__device__ __forceinline__ void ao_rowcol(int f, int T, int &row, int &col) {
    const int c = f & 1, l = (f >> 1) & 63, rest = f >> 7;
    const int kh = rest % (2 * T), I = rest / (2 * T);
    row = 16 * I + (l & 15);
    col = 4 * (2 * kh + c) + (l >> 4);
}

// ---- single-precision operands (mixed-precision formation) -------------------
// v_mfma_f32_16x16x4f32 reads its A and B operands like the FP64 instruction
// but leaves register r of the accumulator holding D[4 (l/16) + r][l%16]
// (rows 4 apart in the FP64 form are adjacent here).  The same operands in
// single precision are stored four k-steps per lane as one float4:
//   flat32(I, kk, l) = ((I T + kk/4) 64 + l) 4 + kk % 4.
__device__ __forceinline__ int ao32_index(int row, int col, int T) {
    const int I = row >> 4, kk = col >> 2, l = (row & 15) | ((col & 3) << 4);
    return ((I * T + (kk >> 2)) * 64 + l) * 4 + (kk & 3);
}
__device__ __forceinline__ void ao32_rowcol(int f, int T, int &row, int &col) {
    const int c = f & 3, l = (f >> 2) & 63, rest = f >> 8;
    const int kq = rest % T, I = rest / T;
    row = 16 * I + (l & 15);
    col = 16 * kq + 4 * c + (l >> 4);
}
// Row order of the single-precision C': within each block of 16 rows, row
// 4 g + r is stored at position 4 r + g.  With C' so permuted, U = C' Xall^T
// comes out of the single-precision accumulator in the FP64 register order,
// so the second product P = Xall U consumes it exactly as in FP64.
__host__ __device__ __forceinline__ int sig16(int row) {
    return (row & ~15) | ((row & 3) << 2) | ((row >> 2) & 3);
}

// ---- the formation products ---------------------------------------------------
// This lane's operand registers of one d x d matrix: a[I][kk] = element of
// row tile I at k-step kk (the A order above).
template <int T>
__device__ __forceinline__ void load_ops(const double2 *__restrict__ M, double (&a)[T][4 * T], int l) {
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int h = 0; h < 2 * T; ++h) {
            const double2 v = M[(I * 2 * T + h) * 64 + l];
            a[I][2 * h] = v.x;
            a[I][2 * h + 1] = v.y;
        }
}
template <int T>
__device__ __forceinline__ void load_ops(const float4 *__restrict__ M, float (&a)[T][4 * T], int l) {
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int q = 0; q < T; ++q) {
            const float4 v = M[(I * T + q) * 64 + l];
            a[I][4 * q] = v.x;
            a[I][4 * q + 1] = v.y;
            a[I][4 * q + 2] = v.z;
            a[I][4 * q + 3] = v.w;
        }
}
// U = C' Xall^T (all tiles, returned as well), then the tiles I <= J of
// P = Xall U.  The accumulator of U's
// tile (I, J), register r, is the B operand of P at k-step 4 I + r (in single
// precision because C' is stored with its rows in the order sig16).
template <int T>
__device__ __forceinline__ void form_p(const double (&xa)[T][4 * T], const double (&ca)[T][4 * T],
                                       so_d4 (&P)[T][T], so_d4 (&U)[T][T]) {
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J) U[I][J] = so_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4 * T; ++kk)
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = 0; J < T; ++J)
                U[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[I][kk], xa[J][kk], U[I][J], 0, 0, 0);
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J) P[I][J] = so_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4 * T; ++kk)
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = I; J < T; ++J)
                P[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[I][kk], U[kk >> 2][J][kk & 3], P[I][J], 0, 0, 0);
}
template <int T>
__device__ __forceinline__ void form_p(const float (&xa)[T][4 * T], const float (&ca)[T][4 * T], so_f4 (&P)[T][T],
                                       so_f4 (&U)[T][T]) {
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J) U[I][J] = so_f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kk = 0; kk < 4 * T; ++kk)
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = 0; J < T; ++J)
                U[I][J] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[I][kk], xa[J][kk], U[I][J], 0, 0, 0);
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J < T; ++J) P[I][J] = so_f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kk = 0; kk < 4 * T; ++kk)
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = I; J < T; ++J)
                P[I][J] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[I][kk], U[kk >> 2][J][kk & 3], P[I][J], 0, 0, 0);
}
// row of P held by register r of a tile's accumulator in lane l (the column
// is 16 J + l % 16)
__device__ __forceinline__ int p_row(const so_d4 &, int I, int r, int l) { return 16 * I + 4 * r + (l >> 4); }
__device__ __forceinline__ int p_row(const so_f4 &, int I, int r, int l) { return 16 * I + 4 * (l >> 4) + r; }

// fz_kernels.hip -- HIP kernels of libfz for gfx950 (CDNA4, wave64).
//
//   fz_dp_*_kernel      count table S[k][v] (completions of a prefix) and the
//                       work table used to cut slices
//   fz_restab_kernel    first element of the last-pair progression per
//                       residue class of the remainder modulo g[d-1]
//   fz_slices_kernel    slice bounds cut to equal work (Sec. 4 bounds)
//   fz_enum_kernel      the walker: bounded lexicographic enumeration with a
//                       count / length-histogram / predicate / store consumer
//   fz_hist_reduce_kernel  sum of the walker workgroups' histogram rows
//   fz_slice_sums_kernel  totals and the slice self-check
//   fz_finalize_kernel  histogram integration, min / max length
//   fz_unrank_kernel    element of a given rank (the fz_unrank entry point)
//   fz_batch_*          the same steps for many queries in one launch each
//
// Layout and notation are described in fz_internal.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fz_internal.h"

namespace {

__device__ __forceinline__ uint64_t sat_add(uint64_t x, uint64_t y)
{
    uint64_t s = x + y;
    return s < x ? ~0ull : s;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FzFastDiv &f)
{
    uint32_t t = __umulhi(f.m, x);
    return (t + ((x - t) >> f.s1)) >> f.s2;
}

// x mod f.d, exact for every x < 2^32.
__device__ __forceinline__ uint32_t fmod32(uint32_t x, const FzFastDiv &f)
{
    return x - fdiv(x, f) * f.d;
}

// A lane's 64-bit value read by the whole wave (a wave-uniform result).
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t uni(uint32_t x)
{
    return __builtin_amdgcn_readfirstlane(x);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane)
{
#pragma unroll
    for (int o = 1; o < FZK_WAVE; o <<= 1) {
        uint32_t t = __shfl_up(v, o, FZK_WAVE);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v, uint32_t lane)
{
#pragma unroll
    for (int o = 1; o < FZK_WAVE; o <<= 1) {
        uint64_t t = __shfl_up(v, o, FZK_WAVE);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

// Sum of a per-lane 64-bit value over the wave, returned to every lane as a
// wave-uniform value.
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (int o = FZK_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, FZK_WAVE);
    return readlane64(v, 0);
}

// S[d-1][v] = [g[d-1] divides v]; rows 0..d-2 are stored.
__device__ __forceinline__ uint64_t table_below(const FzPlan &P, const uint64_t *S, uint32_t k,
                                                uint32_t v)
{
    if (k + 1 == P.d - 1) return (v - fdiv(v, P.div_B) * P.B) == 0 ? 1ull : 0ull;
    return S[(uint64_t)(k + 1) * P.stride + v];
}

// Largest t in [0, v / gk] with Srow[v] - Srow[v - t gk] <= r: the number of
// completions with a_k < t is Srow[v] - Srow[v - t gk] (a telescoping sum of
// the next row), so t is the value of a_k at rank r.  r is reduced in place.
__device__ __forceinline__ uint32_t unrank_level(const uint64_t *Srow, uint32_t v, uint32_t gk,
                                                 uint64_t &r)
{
    const uint64_t sv = Srow[v];
    uint32_t lo = 0, hi = v / gk;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (sv - Srow[v - mid * gk] <= r) lo = mid;
        else hi = mid - 1;
    }
    r -= sv - Srow[v - lo * gk];
    return lo;
}

} // namespace

// ---------------------------------------------------------------------------
// Count and work tables.  S[k][v] = #{(a_k..a_{d-1}) >= 0 : sum_{j>=k} a_j g_j
// = v} satisfies S[k][v] = S[k+1][v] + S[k][v - g_k]: along each chain
// v = c, c + g_k, c + 2 g_k, ... row k is the running sum of row k+1.  The
// work table C models what a wave pays: C[M][v] is the work of one row with
// remainder v (row_work), and C[k][v] = C[k+1][v] + C[k][v - g_k] sums it
// over the subtrees, so slices can be cut to equal work.
// A row is g_k independent chains, each cut into blocks (partial sums, the
// carries, then the final pass): a batch builds a query's rows in one
// workgroup, a single query over the whole chip (a launch per pass).
// Saturating adds: S[0][n] = 2^64-1 flags overflow.
// ---------------------------------------------------------------------------
// Work of the first t lanes (x = 0..t-1) of a row with remainder v: the row
// itself, its 64-lane chunks and its elements.  t = floor(v / G2) + 1 is the
// whole row.  Non-decreasing in t.
__device__ __forceinline__ uint64_t row_work(const FzPlan &P, const uint64_t *SM, uint32_t v,
                                             uint32_t t, const uint64_t *PC)
{
    if (t == 0) return 0;
    if ((P.prune || P.rowtest) && SM[v] == 0) return P.w_skip; // an empty row is not walked
    const uint64_t el = SM[v] - (t * (uint64_t)P.G2 <= v ? SM[v - t * P.G2] : 0);
    // lanes visit all t values of x, or with the pair table only the ones
    // with an element
    const uint64_t lanes =
        P.pair ? PC[v] - (t * (uint64_t)P.G2 <= v ? PC[v - t * P.G2] : 0) : (uint64_t)t;
    // (the packed walk shares chunks between rows: a lane prefix costs a
    // 64th of one)
    const uint64_t chunks = P.pack ? 0 : (lanes + FZK_WAVE - 1) / FZK_WAVE;
    uint64_t w = P.w_row + chunks * P.w_chunk;
    if (P.pack) w += (lanes * P.w_chunk + FZK_WAVE - 1) / FZK_WAVE;
    const uint64_t we = el * P.w_el;
    return (P.w_el && we / P.w_el != el) ? ~0ull : sat_add(w, we);
}

// Running sums along the chains v = c, c + gk, c + 2 gk, ... < len of
// below(v), written to row[v]; in place is allowed (row[v] is written only
// by the thread that read below(v)).  SAT: saturating adds (count tables);
// else wrapping adds (the histogram's difference array, whose entries may be
// negative in two's complement).  The workgroup takes the chains c = c0,
// c0 + cstep, ... (all of them by default): chains are independent, so
// several workgroups can share a row.
template <bool SAT, class Below>
__device__ void chain_scan(uint64_t *row, uint32_t len, uint32_t gk, Below below, uint64_t *part,
                           uint32_t c0 = 0, uint32_t cstep = 1)
{
    const auto add = [](uint64_t a, uint64_t b) { return SAT ? sat_add(a, b) : a + b; };
    const uint32_t T = blockDim.x, tid = threadIdx.x;
    const uint32_t rows = (len - 1) / gk + 1;
    const uint32_t all = gk < len ? gk : len;
    const uint32_t cols = all > c0 ? (all - c0 + cstep - 1) / cstep : 0; // this group's chains
    if (cols == 0) return;
    const uint32_t nb = cols >= T ? 1 : T / cols;
    const uint32_t rpb = (rows + nb - 1) / nb;
    const uint32_t units = cols * nb;
    if (nb > 1) {
        for (uint32_t u = tid; u < units; u += T) {
            const uint32_t c = c0 + (u % cols) * cstep, b = u / cols;
            const uint32_t i1 = min(rows, (b + 1) * rpb);
            uint64_t s = 0;
            // independent loads first, then the dependent sum
            for (uint32_t i = b * rpb; i < i1; i += 8) {
                uint64_t x[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint64_t v = (uint64_t)(i + q) * gk + c;
                    x[q] = (i + q < i1 && v < len) ? below((uint32_t)v) : 0;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) s = add(s, x[q]);
            }
            part[u] = s;
        }
        __syncthreads();
        for (uint32_t c = tid; c < cols; c += T) {
            uint64_t carry = 0;
            for (uint32_t b = 0; b < nb; ++b) {
                const uint64_t t = part[b * cols + c];
                part[b * cols + c] = carry;
                carry = add(carry, t);
            }
        }
        __syncthreads();
    }
    for (uint32_t u = tid; u < units; u += T) {
        const uint32_t c = c0 + (u % cols) * cstep, b = u / cols;
        const uint32_t i1 = min(rows, (b + 1) * rpb);
        uint64_t run = nb > 1 ? part[u] : 0;
        for (uint32_t i = b * rpb; i < i1; i += 8) {
            uint64_t x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint64_t v = (uint64_t)(i + q) * gk + c;
                x[q] = (i + q < i1 && v < len) ? below((uint32_t)v) : 0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint64_t v = (uint64_t)(i + q) * gk + c;
                run = add(run, x[q]);
                if (i + q < i1 && v < len) row[v] = run;
            }
        }
    }
    __syncthreads();
}

// Pair table of a query, after its count table (whole workgroup): a pair
// remainder w is representable when the last pair has a completion,
// S[d-2][w] > 0.  PC[v] counts the representable w <= v with w = v (mod G2);
// PO[r] is where chain r's list starts in PE, PO[nc] the total; PE lists
// each chain's representable remainders in ascending order.
__device__ void pair_table(const FzPlan &P, const uint64_t *S, uint64_t *PC, uint32_t *PE,
                           uint32_t *PO, uint64_t *part)
{
    const uint64_t *Sp = S + (uint64_t)(P.d - 2) * P.stride;
    chain_scan<false>(PC, P.stride, P.G2, [&](uint32_t v) { return Sp[v] ? 1ull : 0ull; }, part);
    const uint32_t T = blockDim.x, tid = threadIdx.x;
    const uint32_t nc = P.G2 < P.stride ? P.G2 : P.stride;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < nc; base += T) {
        const uint32_t r = base + tid;
        uint64_t t = 0;
        if (r < nc) t = PC[r + fdiv(P.n - r, P.div_G2) * P.G2]; // the chain's last entry
        part[tid] = t;
        __syncthreads();
        for (uint32_t o = 1; o < T; o <<= 1) {
            const uint64_t x = tid >= o ? part[tid - o] : 0;
            __syncthreads();
            part[tid] += x;
            __syncthreads();
        }
        if (r < nc) PO[r] = (uint32_t)(carry + part[tid] - t);
        carry += part[T - 1];
        __syncthreads();
    }
    if (tid == 0) PO[nc] = (uint32_t)carry;
    __syncthreads();
    for (uint32_t v = tid; v <= P.n; v += T)
        if (Sp[v]) {
            const uint32_t r = v - fdiv(v, P.div_G2) * P.G2;
            PE[PO[r] + (uint32_t)PC[v] - 1] = v;
        }
    __syncthreads();
}

// All rows of S (k = d-2..0) and of the work table C (k = M..0) for one
// query; called by a whole workgroup of 1024 threads.  PAIR: the
// pair table too, when P.pair.
template <bool PAIR>
__device__ void dp_query(const FzPlan &P, uint64_t *S, uint64_t *C, uint64_t *part, uint64_t *PC,
                         uint32_t *PE, uint32_t *PO)
{
    for (int k = (int)P.d - 2; k >= 0; --k) {
        uint64_t *row = S + (uint64_t)k * P.stride;
        const uint64_t *nxt = S + (uint64_t)(k + 1) * P.stride;
        if (k + 1 == (int)P.d - 1)
            chain_scan<true>(
                row, P.stride, P.g[k],
                [&](uint32_t v) { return (v - fdiv(v, P.div_B) * P.B) == 0 ? 1ull : 0ull; }, part);
        else
            chain_scan<true>(row, P.stride, P.g[k], [&](uint32_t v) { return nxt[v]; }, part);
    }
    if constexpr (PAIR)
        if (P.pair) pair_table(P, S, PC, PE, PO, part);
    const int M = (int)P.d - 3;
    uint64_t *CM = C + (uint64_t)M * P.stride;
    const uint64_t *SM = S + (uint64_t)M * P.stride;
    for (uint32_t v = threadIdx.x; v <= P.n; v += blockDim.x)
        CM[v] = row_work(P, SM, v, fdiv(v, P.div_G2) + 1, PC);
    __syncthreads();
    for (int k = M - 1; k >= 0; --k) {
        uint64_t *row = C + (uint64_t)k * P.stride;
        const uint64_t *nxt = C + (uint64_t)(k + 1) * P.stride;
        chain_scan<true>(row, P.stride, P.g[k], [&](uint32_t v) { return nxt[v]; }, part);
    }
}

// A single query's tables use the whole chip: each row is scanned by
// FZK_DP_UNITS threads, chain c cut into nb blocks of rpb chain steps (unit
// u = block b of chain c, u = b cols + c).  Pass 1 sums each block into part;
// pass 2 adds the sums of the chain's earlier blocks and writes the running
// sums.  BELOW_DIV: the source row is the indicator of g_{d-1} | v (the row
// below the last count-table row), else src[v].
template <bool BELOW_DIV>
__device__ __forceinline__ uint64_t dp_below(const FzPlan &P, const uint64_t *src, uint32_t v)
{
    if constexpr (BELOW_DIV) return (v - fdiv(v, P.div_B) * P.B) == 0 ? 1ull : 0ull;
    else return src[v];
}

template <bool BELOW_DIV>
__global__ void fz_dp_sums_kernel(FzPlan P, const uint64_t *src, uint32_t gk, uint32_t cols,
                                  uint32_t nb, uint32_t rpb, uint64_t *part)
{
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= cols * nb) return;
    const uint32_t c = u % cols, b = u / cols;
    const uint32_t rows = (P.stride - 1) / gk + 1;
    const uint32_t i1 = min(rows, (b + 1) * rpb);
    uint64_t s = 0;
    // independent loads first, then the dependent sum
    for (uint32_t i = b * rpb; i < i1; i += 8) {
        uint64_t x[8];
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) {
            const uint64_t v = (uint64_t)(i + q) * gk + c;
            x[q] = (i + q < i1 && v < P.stride) ? dp_below<BELOW_DIV>(P, src, (uint32_t)v) : 0;
        }
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) s = sat_add(s, x[q]);
    }
    part[u] = s;
}

template <bool BELOW_DIV>
__global__ void fz_dp_apply_kernel(FzPlan P, const uint64_t *src, uint64_t *row, uint32_t gk,
                                   uint32_t cols, uint32_t nb, uint32_t rpb, const uint64_t *part)
{
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= cols * nb) return;
    const uint32_t c = u % cols, b = u / cols;
    const uint32_t rows = (P.stride - 1) / gk + 1;
    const uint32_t i1 = min(rows, (b + 1) * rpb);
    uint64_t run = 0;
    for (uint32_t j = 0; j < b; j += 8) {
        uint64_t x[8];
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) x[q] = j + q < b ? part[(j + q) * cols + c] : 0;
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) run = sat_add(run, x[q]);
    }
    for (uint32_t i = b * rpb; i < i1; i += 8) {
        uint64_t x[8];
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) {
            const uint64_t v = (uint64_t)(i + q) * gk + c;
            x[q] = (i + q < i1 && v < P.stride) ? dp_below<BELOW_DIV>(P, src, (uint32_t)v) : 0;
        }
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) {
            const uint64_t v = (uint64_t)(i + q) * gk + c;
            run = sat_add(run, x[q]);
            if (i + q < i1 && v < P.stride) row[v] = run;
        }
    }
}

// The row of the work table that prices single rows: C[M][v] = row_work.
__global__ void fz_dp_work_kernel(FzPlan P, FzBufs Bf)
{
    const uint32_t M = P.d - 3;
    uint64_t *CM = Bf.C + (uint64_t)M * P.stride;
    const uint64_t *SM = Bf.S + (uint64_t)M * P.stride;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v <= P.n; v += gridDim.x * blockDim.x)
        CM[v] = row_work(P, SM, v, fdiv(v, P.div_G2) + 1, Bf.PC);
}

// The pair table of a single query (one workgroup), after its count table.
__global__ void __launch_bounds__(1024) fz_pair_kernel(FzPlan P, FzBufs Bf)
{
    __shared__ uint64_t part[1024];
    pair_table(P, Bf.S, Bf.PC, Bf.PE, Bf.PO, part);
}

// ---------------------------------------------------------------------------
// Residue table for the last pair (A, B) = (g[d-2], g[d-1]).  For a remainder
// rem = q B + rho the valid a[d-2] are t = t0 + j ord (j >= 0) with
// A t0 == rho (mod B), 0 <= t0 < ord; then a[d-1] = q - E - j delta with
// E = (A t0 - rho) / B.  Classes with gcd(A,B) not dividing rho have no
// element: E = FZK_NONE_E makes a[d-1] negative.  The table is doubled so
// that a lane can index it with rho' = rho + B in [0, 2B) and quotient
// q' = q - 1 without a borrow: entry rho' >= B holds E(rho' - B) - 1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int2 restab_entry(const FzPlan &P, uint32_t i)
{
    const uint32_t rho = i < P.B ? i : i - P.B;
    int2 e;
    if (rho % P.D != 0) {
        e.x = 0;
        e.y = FZK_NONE_E;
    } else {
        const uint64_t t0 = ((uint64_t)(rho / P.D) * P.inv) % P.ord;
        const uint64_t num = (uint64_t)P.A * t0 - rho;
        e.x = (int)t0;
        e.y = (int)(num / P.B);
        if (i >= P.B) e.y -= 1;
    }
    return e;
}

__global__ void fz_restab_kernel(FzPlan P, FzBufs Bf)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2 * P.B) Bf.restab[i] = restab_entry(P, i);
}

// ---------------------------------------------------------------------------
// Slice bounds, cut by work.  Lane prefixes a[0..M] in lex order carry the
// work of the wave that walks them (row_work).  Boundary j (0 <= j < W) is
// the prefix at work rank floor(j Wtot / W): found level by level in the work
// table for the row prefix a[0..M-1], then inside the row on the row_work of
// its first t lanes.  Wtot covers the prefixes up to the one that holds
// element rank N' - 1, N' = min(|Z|, max_tuples).  Slice j walks prefixes
// [bound j, bound j+1); base[j] is the element rank of its first element.
// Boundary W is open (sentinel).  Thread 0 also resets the control block.
// ---------------------------------------------------------------------------
// Boundary j of a query cut into W slices: writes its prefix a[0..M] (or the
// sentinel) to out and returns the element rank of its first element.
__device__ uint64_t slice_bound(const FzPlan &P, const uint64_t *S, const uint64_t *C, uint32_t W,
                                uint32_t j, uint32_t *out, const uint64_t *PC)
{
    const uint32_t M = P.d - 3;
    const uint64_t N = S[P.n];
    const bool ovf = (N == ~0ull) || (C[P.n] == ~0ull);
    const uint64_t Np = ovf ? 0 : (N < P.max_tuples ? N : P.max_tuples);
    if (j >= W || Np == 0) {
        out[0] = FZK_SENTINEL;
        return Np;
    }
    const uint64_t *SM = S + (uint64_t)M * P.stride;
    uint64_t Wtot;
    if (Np == N) {
        Wtot = C[P.n];
    } else {
        // work of the rows before the one that holds element rank Np-1, plus
        // that row up to and including the lane holding it
        uint64_t r = Np - 1, acc = 0;
        uint32_t v = P.n;
        for (uint32_t k = 0; k < M; ++k) {
            const uint64_t *Ck = C + (uint64_t)k * P.stride;
            const uint32_t t = unrank_level(S + (uint64_t)k * P.stride, v, P.g[k], r);
            acc += Ck[v] - Ck[v - t * P.g[k]];
            v -= t * P.g[k];
        }
        const uint32_t x = unrank_level(SM, v, P.G2, r);
        Wtot = acc + row_work(P, SM, v, x + 1, PC);
    }
    // work rank of bound j: W equal parts, or, with a host share, W - T
    // equal parts of the device's work and T of the host's.  guided: the
    // last W/4 slices take a quarter of the work of each of the others, so
    // that the slices still walked after the cursor has run out are short.
    uint64_t rc;
    const uint32_t T = P.host_slices;
    if (T == 0 && P.guided && W >= 64) {
        const uint64_t L = W / 4, U = 4 * (uint64_t)(W - L) + L;
        const uint64_t u = j <= W - L ? 4 * (uint64_t)j : 4 * (uint64_t)(W - L) + (j - (W - L));
        rc = (Wtot / U) * u + ((Wtot % U) * u) / U;
    } else if (T == 0) {
        rc = (Wtot / W) * j + ((Wtot % W) * j) / W;
    } else {
        const uint32_t Wd = W - T;
        const uint64_t Wh = (uint64_t)((double)Wtot * (P.host_ppm * 1e-6));
        const uint64_t Wdev = Wtot - Wh;
        rc = j <= Wd ? (Wdev / Wd) * j + ((Wdev % Wd) * j) / Wd
                     : Wdev + (Wh / T) * (j - Wd) + ((Wh % T) * (j - Wd)) / T;
    }
    uint64_t base = 0;
    uint32_t v = P.n;
    for (uint32_t k = 0; k < M; ++k) {
        const uint64_t *Sk = S + (uint64_t)k * P.stride;
        const uint32_t t = unrank_level(C + (uint64_t)k * P.stride, v, P.g[k], rc);
        base += Sk[v] - Sk[v - t * P.g[k]];
        out[k] = t;
        v -= t * P.g[k];
    }
    // inside the row: largest t in [0, v / G2] whose first t lanes fit in rc
    uint32_t lo = 0, hi = v / P.G2;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (row_work(P, SM, v, mid, PC) <= rc) lo = mid;
        else hi = mid - 1;
    }
    out[M] = lo;
    base += SM[v] - SM[v - lo * P.G2];
    return base;
}

// Slices of a single query: W = P.n_slices, or fewer when the query's whole
// modelled work C[0][n] is small, so that every slice carries at least
// P.min_slice_work (a small query then occupies a few waves briefly instead
// of every wave of the chip).  Every thread computes the same value.
__device__ __forceinline__ uint32_t cut_slices(const FzPlan &P, const uint64_t *C)
{
    if (P.min_slice_work == 0 || P.host_slices) return P.n_slices;
    const uint64_t k = C[P.n] / P.min_slice_work + 1;
    return k < P.n_slices ? (uint32_t)k : P.n_slices;
}

__global__ void fz_slices_kernel(FzPlan P, FzBufs Bf)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t W = cut_slices(P, Bf.C);
    if (j == 0) {
        const uint64_t N = Bf.S[P.n];
        const bool ovf = (N == ~0ull) || (Bf.C[P.n] == ~0ull);
        FzCtl *c = Bf.ctl;
        c->cursor = 0;
        c->found = 0;
        c->status = ovf ? FZS_OVERFLOW : 0u;
        c->slices = W;
        c->total = N;
        c->count = 0;
        c->rows = 0;
        c->prefixes = 0;
        c->written = 0;
    }
    const uint32_t Wall = W + P.host_slices; // and the host's slices after the device's
    if (j > Wall) return;
    // a predicate's walkers may stop before taking every slice: slices
    // nobody walks must read as empty in the totals
    if (j < W) Bf.recs[j] = FzSliceRec{};
    Bf.base[j] = slice_bound(P, Bf.S, Bf.C, Wall, j, Bf.bounds + (uint64_t)j * (P.d - 2), Bf.PC);
}

// ---------------------------------------------------------------------------
// The walker.  Within a slice the row prefix a[0..M-1] is a wave-uniform
// odometer in ascending lex order (scalar registers); a row is cut into
// chunks of 64 consecutive values of the lane coordinate x = a[M]; each lane
// solves its last pair from the residue table and then steps its progression
// of elements one candidate at a time (the modulo skip of Sec. 3.2.4:
// a[d-2] += ord, a[d-1] -= delta), the step ending at the first candidate
// with a[d-1] < 0.  The consumer sees every element.
//
// walk_slice walks one slice [b0, b1) for one wave.  MAXM bounds the row
// depth M (M == MAXM in the single-query kernel, where it is a compile-time
// constant; the batch kernel passes each query's own M <= MAXM).
// ---------------------------------------------------------------------------
struct WalkIO {
    const int2 *ltab;   // residue table staged in LDS (TLDS)
    const int2 *gtab;   // residue table in global memory (!TLDS)
    uint64_t *wbins;    // LDS histogram (difference array), 64-bit bins: the workgroup's
                        // (single query) or this wave's (batch)
    uint32_t *wbins32;  // ... 32-bit bins (batches: every bin of an item stays below 2^31)
    uint32_t *wbins32l; // single query: this lane's copy of the wave's 32-bit bins (bin b at
                        // wbins32l[b << w32k])
    uint32_t w32k;
    uint64_t *gbins;    // the global histogram (bins not in LDS)
    uint32_t *found;    // predicate flag (early exit)
    uint32_t *out;      // store destination, row-major [.][d_user]
    uint64_t *s_incl;   // store scratch of this wave: scan, t0, ad0, rows
    uint32_t *s_t0, *s_ad0, *s_stage;
    uint32_t *s_x;      // store scratch: each lane's x, when not consecutive
    const uint64_t *S;  // count table, for skipping empty subtrees (P.prune)
    const uint64_t *PC; // pair table (P.pair): representable remainders up to v, per chain
    const uint32_t *PE; //   the representable remainders, ascending per chain
    const uint32_t *PO; //   where each chain's list starts in PE
    const uint64_t *TO; // trailing tables (P.trail): offsets and triples
    const uint32_t *TT;
    uint64_t trail_m;   //   full rows with remainder < trail_m take them
};

struct WalkOut {
    uint64_t elements, rows, prefixes;
};

// One run of a lane: cnt elements with lengths len0, len0 + step, ...
// Recorded in the histogram's strided difference array (stride |step|): +1
// at the run's shortest length and -1 one stride past its longest; with
// step 0 all cnt elements have length len0.  Bins wrap, so negative entries
// are two's complement: 64-bit bins, or 32-bit ones in a batch, where a bin
// moves by at most the elements of one work item (< 2^30, checked on the
// host) and is flushed, sign-extended, after every item.  H32 (a single
// query): the run goes to the wave's own 32-bit bins, io.wbins32.
template <bool FIXED, bool H32 = false>
__device__ __forceinline__ void hist_run(const FzPlan &P, const WalkIO &io, uint32_t len0,
                                         uint32_t cnt, int32_t step)
{
    if constexpr (FIXED) {
        // A single query's bins (LDS or global, 64-bit) have one spare bin
        // at index nbins that takes the -1 of a run ending past the last bin
        // (and of every run when step is 0), so both adds are unconditional.
        const uint32_t mag = step < 0 ? (uint32_t)-step : (uint32_t)step;
        const uint32_t lo = step < 0 ? len0 - (cnt - 1) * mag : len0;
        const uint32_t hi0 = lo + cnt * mag;
        const uint32_t hi = (mag != 0 && hi0 < P.nbins) ? hi0 : P.nbins;
        const uint64_t inc = mag != 0 ? 1ull : (uint64_t)cnt;
        if (H32) { // the lane's copy of the wave's 32-bit bins
            __hip_atomic_fetch_add(&io.wbins32l[lo << io.w32k], (uint32_t)inc, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(&io.wbins32l[hi << io.w32k], 0xFFFFFFFFu, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if (P.hist_in_lds) { // the workgroup's bins
            __hip_atomic_fetch_add(&io.wbins[lo], inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(&io.wbins[hi], ~0ull, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            __hip_atomic_fetch_add(&io.gbins[lo], inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&io.gbins[hi], ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    uint32_t lo = len0, inc = cnt;
    uint64_t hi = ~0ull;
    if (step != 0) {
        const uint32_t mag = step > 0 ? (uint32_t)step : (uint32_t)-step;
        if (step < 0) lo = len0 - (cnt - 1) * mag;
        hi = (uint64_t)lo + (uint64_t)cnt * mag;
        inc = 1;
    }
    if (P.hist_in_lds == 2) {
        atomicAdd(&io.wbins32[lo], inc);
        if (hi < P.nbins) atomicAdd(&io.wbins32[hi], 0xFFFFFFFFu);
    } else if (P.hist_in_lds) {
        atomicAdd((unsigned long long *)&io.wbins[lo], (unsigned long long)inc);
        if (hi < P.nbins) atomicAdd((unsigned long long *)&io.wbins[hi], ~0ull);
    } else {
        atomicAdd((unsigned long long *)&io.gbins[lo], (unsigned long long)inc);
        if (hi < P.nbins) atomicAdd((unsigned long long *)&io.gbins[hi], ~0ull);
    }
}

// Moves the row odometer a[0..M-1] (remainders rr) to the first row, at or
// after the current one and not past the end prefix e, whose every level has
// a completion: S[k+1][rr[k+1]] > 0 for all k < M.  An empty subtree is
// skipped as a whole: the wave tests 64 siblings at once (lane i takes
// a[k] + i) and jumps to the first non-empty one, or moves on to the next
// prefix of a shallower level when none is left.  Levels < chk are known to
// be non-empty.  Returns false when the slice has no such row left.
template <int MAXM>
__device__ __forceinline__ bool skip_empty(const FzPlan &P, const uint32_t M, const uint64_t *S,
                                           uint32_t *a, uint32_t *rr, const uint32_t *e,
                                           bool end_open, int &chk, bool &moved, uint32_t lane)
{
    auto advance = [&](int kk, uint32_t j) {
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            if (k == kk) {
                a[k] += j;
                rr[k + 1] -= j * P.g[k];
            } else if (k > kk) {
                a[k] = 0;
                rr[k + 1] = rr[k];
            }
        }
    };
    for (;;) {
        int kz = -1;
#pragma unroll
        for (int k = 0; k < MAXM; ++k)
            if (k < (int)M && k >= chk && kz < 0) {
                const uint64_t c = S[(uint64_t)(k + 1) * P.stride + rr[k + 1]];
                if ((uni((uint32_t)c) | uni((uint32_t)(c >> 32))) == 0) kz = k;
            }
        if (kz < 0) {
            chk = (int)M;
            return true;
        }
        moved = true;
        bool pe = !end_open; // a[0..kz-1] is the end prefix's: a[kz] <= e[kz]
        uint32_t gk = 0, ak = 0, rk = 0, ek = 0;
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            if (k < kz) pe = pe && a[k] == e[k];
            if (k == kz) {
                gk = P.g[k];
                ak = a[k];
                rk = rr[k + 1];
                ek = e[k];
            }
        }
        const int64_t v = (int64_t)rk - (int64_t)lane * gk;
        const bool in = v >= 0 && (!pe || ak + lane <= ek);
        const bool nz = in && S[(uint64_t)(kz + 1) * P.stride + (uint64_t)v] != 0;
        const uint64_t m = __ballot(nz);
        if (m) {
            advance(kz, (uint32_t)__builtin_ctzll(m));
            chk = kz + 1;
            continue;
        }
        // all 64 were empty: go on at a[kz] + 64 if that sibling exists (its
        // remainder is >= 0 and, under the end prefix, it is <= e[kz])
        const bool more = (int64_t)rk - (int64_t)FZK_WAVE * gk >= 0 && (!pe || ak + FZK_WAVE <= ek);
        if (more) {
            advance(kz, FZK_WAVE);
            chk = kz;
            continue;
        }
        if (pe) return false; // the end prefix bounds this level: nothing is left
        // nothing under a[0..kz-1]: the next prefix of a shallower level (it
        // cannot pass the end, which lies after this whole subtree)
        int kk = -1;
#pragma unroll
        for (int k = 0; k < MAXM; ++k)
            if (k < kz && rr[k + 1] >= P.g[k]) kk = k;
        if (kk < 0) return false;
        advance(kk, 1);
        chk = kk;
    }
}

// The element loop of a dense walk: two candidate steps per trip (ad >= 0,
// ad >= delta: one element each), then ad -= 2 delta, while some lane's next
// step is valid.  Written out so that each trip is five vector instructions
// and one branch: the validity test of a step is the carry into the count.
// Every lane of the wave must be active.
__device__ __forceinline__ void count_steps(uint32_t &cnt, int32_t &ad, int32_t delta,
                                            int32_t delta2)
{
    asm volatile("v_cmp_le_i32 vcc, 0, %1\n"
                 "s_cbranch_vccz 2f\n"
                 "1:\n"
                 "v_addc_co_u32 %0, vcc, 0, %0, vcc\n"
                 "v_cmp_le_i32 vcc, %2, %1\n"
                 "v_addc_co_u32 %0, vcc, 0, %0, vcc\n"
                 "v_subrev_u32 %1, %3, %1\n"
                 "v_cmp_le_i32 vcc, 0, %1\n"
                 "s_cbranch_vccnz 1b\n"
                 "2:\n"
                 : "+v"(cnt), "+v"(ad)
                 : "s"(delta), "s"(delta2)
                 : "vcc");
}

// FIXED: M == MAXM (a compile-time depth: the single-query walker), which
// allows the row fast paths below without per-level selects.
// CDV: the variant walk of the block walker (common-divisor skip over the
// last two and three generators, Sec. 3.2.4, and each lane's run counted in
// closed form): neighbouring lanes are sx apart in x and block rows sy apart.
// PACK: the packed walk of short rows (count, histogram, predicate): the lane
// prefixes of up to 64 rows of the deepest row level are laid end to end and
// walked 64 at a time, so that a chunk is not one row's few prefixes.  (With
// no row level, M = 0, the one row is walked alone.)  H32: histogram runs
// go to the wave's 32-bit bins (io.wbins32 set).
template <int MAXM, int MODE, bool TLDS, bool PRUNE, bool PAIR, bool FIXED, bool CDV = false,
          bool PACK = false, bool H32 = false>
__device__ __forceinline__ WalkOut walk_slice(const FzPlan &P, const uint32_t M,
                                              const uint32_t *b0, const uint32_t *b1,
                                              uint64_t rank, const WalkIO &io, uint32_t lane)
{
    // The lanes of a chunk are G2s = G2 sx apart in remainder (sx = 1 but in
    // the variant walk).  lane * G2s = lq * B + lr (exact whenever the lane
    // is active).  A lane reads the doubled residue table at rho' = Pc + (B -
    // lr) with quotient q' = Qc - (lq + 1): no borrow to propagate.
    const uint32_t sx = CDV ? P.cd_sx : 1u;
    const uint32_t G2s = P.G2 * sx; // < 2^31 (checked on the host)
    const uint64_t lg = (uint64_t)lane * G2s;
    const uint32_t lq1 = (uint32_t)(lg / P.B) + 1;
    const uint32_t lr2 = P.B - (uint32_t)(lg % P.B);
    // 64 G2s = c64q B + c64r: the step of a chunk's remainder (c64q wraps
    // only when no second chunk fits in a row, and is then unused)
    const uint32_t g2q = fdiv(G2s, P.div_B);
    const uint32_t g2r64 = (G2s - g2q * P.B) * FZK_WAVE; // < 64 B <= 2^30
    const uint32_t c64r0q = fdiv(g2r64, P.div_B);
    const uint32_t c64q = g2q * FZK_WAVE + c64r0q;
    const uint32_t c64r = g2r64 - c64r0q * P.B;
    const uint32_t len_step = P.ord - P.delta;
    const int32_t delta = (int32_t)P.delta;
    const int32_t delta2 = 2 * delta; // two candidate steps
    // lengths are < 2^31, so a target beyond 32 bits matches none
    const uint32_t target = P.target_len >> 32 ? FZK_SENTINEL : (uint32_t)P.target_len;
    // per-lane element counters: a chunk adds at most n + 1 per lane to the
    // 32-bit counter, which is folded into the 64-bit one per chunk
    uint64_t lane_el = 0;
    uint32_t lane_pref = 0;
    uint64_t lane_pref64 = 0; // lane prefixes of the rows of the block walk
    uint64_t n_trail = 0;     // elements of rows counted from the count table
    // BLOCKS: a compile-time depth and no row skipping (see the block walk)
    constexpr bool BLOCKS = FIXED && !PRUNE && !PAIR && !PACK && MAXM > 0;
    static_assert(!PACK || (MAXM > 0 && !PAIR && !CDV && MODE != FZM_STORE),
                  "the packed walk serves order-free consumers");
    uint64_t n_el = 0, n_rows = 0;
    if (uni(b0[0]) != FZK_SENTINEL) {
        uint32_t a[MAXM > 0 ? MAXM : 1];
        uint32_t e[MAXM > 0 ? MAXM : 1];
        uint32_t rr[MAXM + 1]; // rr[k]: remainder after a[0..k-1]; constant past M
        rr[0] = P.n;
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            if (k < (int)M) {
                a[k] = uni(b0[k]);
                rr[k + 1] = rr[k] - a[k] * P.g[k];
            } else {
                a[k] = 0;
                rr[k + 1] = rr[k];
            }
        }
        int32_t xs = (int32_t)uni(b0[M]);
        const bool end_open = uni(b1[0]) == FZK_SENTINEL;
        int32_t xe = 0;
#pragma unroll
        for (int k = 0; k < MAXM; ++k) e[k] = 0;
        if (!end_open) {
#pragma unroll
            for (int k = 0; k < MAXM; ++k)
                if (k < (int)M) e[k] = uni(b1[k]);
            xe = (int32_t)uni(b1[M]);
        }
        uint32_t plen = 0;
#pragma unroll
        for (int k = 0; k < MAXM; ++k) plen += a[k];
        int chk = 0; // skip_empty: levels < chk known to have elements
        // FIXED: whether the levels above the deepest equal the end prefix's,
        // recomputed only where those levels change
        auto upper_equal = [&]() -> bool {
            bool u = !end_open;
#pragma unroll
            for (int k = 0; k + 1 < MAXM; ++k) u = u && a[k] == e[k];
            return u;
        };
        bool upper_eq = FIXED ? upper_equal() : false;
        bool done = false;
        // One chunk of lane prefixes: lane l has x = xl, the first valid
        // a[d-2] = t0 and a[d-1] = ad0 there (-1: no element).  For the
        // store, the x of position j's owner is xbase + j, or s_x[j] when
        // the lanes' x are not consecutive.  Returns true to stop the walk.
        auto consume = [&](const uint32_t xl, const uint32_t t0, int32_t ad0, const int32_t xbase,
                           const bool x_in_lds) -> bool {
            uint32_t cnt = 0;
            if constexpr (MODE == FZM_COUNT) {
                // two candidate steps per trip; a trip runs while some
                // lane's next step is valid (no trip that finds nothing).
                // Dense walks enter the loop at once (almost every chunk has
                // an element); the others test first.
                int32_t ad = ad0;
                if constexpr (CDV) { // the run's length in closed form
                    cnt = ad0 >= 0 ? fdiv((uint32_t)ad0, P.div_delta) + 1u : 0u;
                } else if constexpr (BLOCKS || PACK) {
                    count_steps(cnt, ad, delta, delta2);
                } else if (__ballot(ad >= 0)) {
                    do {
                        cnt += ad >= 0 ? 1u : 0u;
                        cnt += ad >= delta ? 1u : 0u;
                        ad -= delta2;
                    } while (__ballot(ad >= 0));
                }
                lane_el += cnt;
            } else if constexpr (MODE == FZM_HIST) {
                // The lane's elements are counted one by one as in the
                // count consumer; their lengths step by len_step, so the
                // run is then recorded as a strided difference (finalize
                // integrates along the stride).
                int32_t ad = ad0;
                if constexpr (CDV) { // the run's length in closed form
                    cnt = ad0 >= 0 ? fdiv((uint32_t)ad0, P.div_delta) + 1u : 0u;
                } else if constexpr (BLOCKS || PACK) {
                    count_steps(cnt, ad, delta, delta2);
                } else if (__ballot(ad >= 0)) {
                    do {
                        cnt += ad >= 0 ? 1u : 0u;
                        cnt += ad >= delta ? 1u : 0u;
                        ad -= delta2;
                    } while (__ballot(ad >= 0));
                }
                lane_el += cnt;
                if (cnt) {
                    const uint32_t len0 = plen + xl + t0 + (uint32_t)ad0;
                    hist_run<FIXED, H32>(P, io, len0, cnt, (int32_t)len_step);
                }
            } else if constexpr (MODE == FZM_EXISTS) {
                // each element's length is compared with the target; the
                // wave looks at the lanes' verdicts once per chunk
                int32_t ad = ad0;
                uint32_t len = plen + xl + t0 + (uint32_t)ad0;
                bool hit = false;
                if (BLOCKS || __ballot(ad >= 0)) {
                    do {
                        const bool c0 = ad >= 0;
                        const bool c1 = ad >= delta;
                        cnt += c0 ? 1u : 0u;
                        cnt += c1 ? 1u : 0u;
                        hit = hit || (c0 && len == target) || (c1 && len + len_step == target);
                        ad -= delta2;
                        len += 2 * len_step;
                    } while (__ballot(ad >= 0));
                }
                lane_el += cnt;
                if (__ballot(hit)) {
                    __hip_atomic_store(io.found, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    return true;
                }
            } else { // FZM_STORE
                uint64_t L = 0;
                if (ad0 >= 0) L = fdiv((uint32_t)ad0, P.div_delta) + 1;
                const uint64_t incl = wave_incl_scan64(L, lane);
                const uint64_t T = readlane64(incl, FZK_WAVE - 1);
                io.s_incl[lane] = incl;
                io.s_t0[lane] = t0;
                io.s_ad0[lane] = (uint32_t)ad0;
                if (x_in_lds) io.s_x[lane] = xl;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // Rows are produced 64 at a time (lane = position in the
                // chunk's output), staged in LDS as one contiguous block
                // and written out as consecutive dwords: every store
                // instruction covers 256 bytes.
                const uint64_t lim = P.max_tuples;
                const uint32_t du = P.d_user;
                for (uint64_t p0 = 0; p0 < T && rank + p0 < lim; p0 += FZK_WAVE) {
                    const uint64_t left = T - p0 < lim - rank - p0 ? T - p0 : lim - rank - p0;
                    const uint32_t nb = left < FZK_WAVE ? (uint32_t)left : FZK_WAVE;
                    const uint64_t p = p0 + lane;
                    if (lane < nb) {
                        uint32_t j = 0;
#pragma unroll
                        for (uint32_t st = FZK_WAVE / 2; st >= 1; st >>= 1)
                            if (io.s_incl[j + st - 1] <= p) j += st;
                        const uint32_t k = (uint32_t)(p - (j ? io.s_incl[j - 1] : 0ull));
                        // coordinates a[0..M-1], x, t, ad; the first pad
                        // (virtual) coordinates are not output
                        uint32_t *st_row = io.s_stage + lane * du;
#pragma unroll
                        for (int q = 0; q < MAXM; ++q)
                            if (q < (int)M && (uint32_t)q >= P.pad) st_row[q - P.pad] = a[q];
                        if (M >= P.pad)
                            st_row[M - P.pad] = x_in_lds ? io.s_x[j] : (uint32_t)xbase + j;
                        if (M + 1 >= P.pad) st_row[M + 1 - P.pad] = io.s_t0[j] + k * P.ord;
                        st_row[M + 2 - P.pad] = io.s_ad0[j] - k * P.delta;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    uint32_t *dst = io.out + (rank + p0) * du;
                    const uint32_t words = nb * du;
                    for (uint32_t i = lane; i < words; i += FZK_WAVE) dst[i] = io.s_stage[i];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (rank < lim) n_el += (T < lim - rank) ? T : (lim - rank);
                rank += T;
                if (rank >= lim) return true;
            }
            return false;
        };

        // Store from the trailing tables: the row a[0..M-1] with remainder Rr
        // gets the triples of Z(Rr), 64 rows at a time staged in LDS and
        // written as consecutive words.  Returns true at the store's limit.
        auto copy_row = [&](const uint32_t Rr) -> bool {
            const uint64_t o0 = readlane64(io.TO[Rr], 0), o1 = readlane64(io.TO[Rr + 1], 0);
            const uint64_t cnt = o1 - o0;
            const uint64_t lim = P.max_tuples;
            const uint32_t du = P.d_user;
            for (uint64_t p0 = 0; p0 < cnt && rank + p0 < lim; p0 += FZK_WAVE) {
                const uint64_t left = cnt - p0 < lim - rank - p0 ? cnt - p0 : lim - rank - p0;
                const uint32_t nb2 = left < FZK_WAVE ? (uint32_t)left : FZK_WAVE;
                if (lane < nb2) {
                    const uint32_t *tr = io.TT + 3 * (o0 + p0 + lane);
                    uint32_t *st_row = io.s_stage + lane * du;
#pragma unroll
                    for (int q = 0; q < MAXM; ++q) st_row[q] = a[q]; // d >= 4: no virtual coordinate
                    st_row[MAXM] = tr[0];
                    st_row[MAXM + 1] = tr[1];
                    st_row[MAXM + 2] = tr[2];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                uint32_t *dst = io.out + (rank + p0) * du;
                const uint32_t words = nb2 * du;
                for (uint32_t i = lane; i < words; i += FZK_WAVE) dst[i] = io.s_stage[i];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (rank < lim) n_el += (cnt < lim - rank) ? cnt : (lim - rank);
            rank += cnt;
            return rank >= lim;
        };

        // BLOCKS (a compile-time depth, no row skipping): the rows of the
        // deepest row level are prepared up to 64 at a time, one per lane --
        // the row's last x and its first chunk's remainder split Rc = Qc B +
        // Pc -- and walked one by one, each read with readlane, so a row
        // costs the scalar unit only its loop step.  Within a row each lane
        // keeps its own table index rho = Pc + lr2 and quotient q = Qc - lq1
        // and steps them by 64 G2 per chunk (a borrow when rho drops below
        // lr2): the chunk loop is vector work but for its one branch.
        if constexpr (BLOCKS) {
            const uint32_t gy = P.g[MAXM > 0 ? MAXM - 1 : 0];
            const uint32_t sy = CDV ? P.cd_sy : 1u;
            // the chunk step of the table offsets, and 8 B kept in a vector
            // register (it is added under a per-lane condition every chunk)
            const uint32_t c64r8 = c64r * 8u, lr2_8 = lr2 * 8u;
            uint32_t vB8 = P.B * 8u;
            asm volatile("" : "+v"(vB8));
            for (;;) {
                uint32_t ay = a[MAXM - 1];
                uint32_t R0 = rr[MAXM];
                if constexpr (CDV) {
                    // the first row at or after ay whose remainder is a
                    // multiple of D3: y = ay + dy with dy (gy / e3) = (R0 mod
                    // D3) / e3 (mod sy); none when e3 does not divide R0
                    const uint32_t r3 = fmod32(R0, P.div_D3);
                    const uint32_t q3 = fdiv(r3, P.div_e3);
                    bool any = r3 == q3 * P.cd_e3;
                    const uint32_t dy = any ? fmod32(q3 * P.cd_inv3, P.div_sy) : 0u;
                    any = any && (uint64_t)dy * gy <= R0 && (!upper_eq || ay + dy <= e[MAXM - 1]);
                    if (!any) {
                        // nothing left on this level: the slice's end when its
                        // end prefix is here, else the next prefix above
                        if (upper_eq) break;
                        int kk = -1;
#pragma unroll
                        for (int k = 0; k + 1 < MAXM; ++k)
                            if (rr[k + 1] >= P.g[k]) kk = k;
                        if (kk < 0) break;
#pragma unroll
                        for (int k = 0; k < MAXM; ++k) {
                            if (k == kk) {
                                a[k] += 1;
                                rr[k + 1] -= P.g[k];
                            } else if (k > kk) {
                                a[k] = 0;
                                rr[k + 1] = rr[k];
                            }
                        }
                        plen = 0;
#pragma unroll
                        for (int k = 0; k < MAXM; ++k) plen += a[k];
                        upper_eq = upper_equal();
                        xs = 0;
                        continue;
                    }
                    if (dy) xs = 0; // the slice's start row had no element
                    ay += dy;
                    R0 -= dy * gy;
                    plen += dy;
                    a[MAXM - 1] = ay;
                    rr[MAXM] = R0;
                }
                // rows y = ay + lane sy while in the set and in the slice
                const uint64_t off = (uint64_t)lane * sy * gy;
                bool in = off <= R0;
                if (upper_eq) in = in && ay + lane * sy <= e[MAXM - 1];
                const uint32_t nb = (uint32_t)__builtin_popcountll(__ballot(in));
                // the slice's end row is the block's last row; no row of the
                // slice is left after the block
                const bool end_here = upper_eq && ay + (nb - 1) * sy == e[MAXM - 1];
                const bool blast = upper_eq && ay + nb * sy > e[MAXM - 1];
                const uint32_t R = R0 - (uint32_t)off; // meaningful for lanes in
                uint32_t x0 = lane == 0 ? (uint32_t)xs : 0u;
                bool has = in;
                if constexpr (CDV) {
                    // the row's first x at or after x0 with x G2 = R (mod D)
                    const uint32_t r2 = fmod32(R, P.div_D);
                    const uint32_t q2 = fdiv(r2, P.div_e2);
                    has = has && r2 == q2 * P.cd_e2;
                    const uint32_t xst = fmod32(q2 * P.cd_inv2, P.div_sx);
                    x0 += fmod32(xst + sx - fmod32(x0, P.div_sx), P.div_sx);
                }
                const int32_t xlast =
                    (end_here && lane + 1 == nb) ? xe - 1 : (int32_t)fdiv(R, P.div_G2);
                // the row's lane prefixes x0, x0 + sx, .., up to xlast (rows of
                // a stopped walk count in full)
                // rowtest: a row whose remainder the count table gives no
                // completion has no element (one vector load tests the
                // block's rows)
                if (P.rowtest && has) has = io.S[(uint64_t)MAXM * P.stride + R] != 0;
                const int32_t v_np =
                    has && xlast >= (int32_t)x0
                        ? (CDV ? (int32_t)fdiv((uint32_t)(xlast - (int32_t)x0), P.div_sx)
                               : xlast - (int32_t)x0) + 1
                        : 0;
                lane_pref64 += (uint32_t)v_np;
                const uint32_t v_x0 = x0;
                const uint32_t v_Rc = R - x0 * P.G2;
                const uint32_t v_Qc = fdiv(v_Rc, P.div_B);
                const uint32_t v_Pc = v_Rc - v_Qc * P.B;
                const uint32_t plen0 = plen;
                // the block's rows that have lane prefixes, in order
                uint64_t rows_left = __ballot(v_np > 0);
                uint32_t j = 0;
                while (rows_left) {
                    j = (uint32_t)__builtin_ctzll(rows_left);
                    rows_left &= rows_left - 1;
                    const int32_t np = (int32_t)__builtin_amdgcn_readlane((uint32_t)v_np, j);
                    const uint32_t Qc = __builtin_amdgcn_readlane(v_Qc, j);
                    const uint32_t Pc = __builtin_amdgcn_readlane(v_Pc, j);
                    // the count does not look at x
                    const int32_t xf =
                        MODE == FZM_COUNT ? 0
                                          : (CDV ? (int32_t)__builtin_amdgcn_readlane(v_x0, j)
                                                 : (j == 0 ? xs : 0));
                    a[MAXM - 1] = ay + j * sy;
                    plen = plen0 + j * sy;
                    if constexpr (MODE == FZM_EXISTS) {
                        const uint32_t f = __hip_atomic_load(io.found, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                        if (uni(f)) {
                            done = true;
                            break;
                        }
                    }
                    if constexpr ((MODE == FZM_COUNT || MODE == FZM_STORE) && !CDV) {
                        // trailing-index tables: a full row (not the slice's
                        // first row begun mid-way, nor its last) with a small
                        // remainder takes Z(R, (G2, A, B)) at once
                        if (P.trail && (j != 0 || xs == 0) && !(end_here && j + 1 == nb)) {
                            const uint32_t Rr = __builtin_amdgcn_readlane(R, j);
                            if constexpr (MODE == FZM_COUNT) {
                                const uint64_t z = io.S[(uint64_t)(P.d - 3) * P.stride + Rr];
                                n_trail += readlane64(z, 0);
                                continue;
                            } else {
                                if ((uint64_t)Rr < io.trail_m) {
                                    if (copy_row(Rr)) {
                                        done = true;
                                        break;
                                    }
                                    continue;
                                }
                            }
                        }
                    }
                    // the lane's table entry as a byte offset: rho * 8, rho in
                    // [lr2, lr2 + B), inside the 2B table
                    uint32_t off = (Pc + lr2) * 8u;
                    int32_t q = (int32_t)(Qc - lq1);
                    int32_t c = xf;
                    int32_t left = np - 1;
                    // Full chunks: every lane has an x.  An active lane's
                    // first candidate is above -delta - 1, so its run needs
                    // no clamp; the last chunk's lanes past the row's end get
                    // -1 (their quotient is meaningless).
                    for (; left >= FZK_WAVE - 1; left -= FZK_WAVE, c += FZK_WAVE * (int32_t)sx) {
                        const int2 ent = TLDS ? *(const int2 *)((const char *)io.ltab + off)
                                              : *(const int2 *)((const char *)io.gtab + off);
                        if (consume((uint32_t)c + lane * sx, (uint32_t)ent.x, q - ent.y, c, false)) {
                            done = true;
                            break;
                        }
                        off -= c64r8;
                        q -= (int32_t)c64q;
                        if ((int32_t)off < (int32_t)lr2_8) {
                            off += vB8;
                            q -= 1;
                        }
                    }
                    if (!done && left >= 0) {
                        const bool active = (int32_t)lane <= left;
                        const int2 ent = TLDS ? *(const int2 *)((const char *)io.ltab + off)
                                              : *(const int2 *)((const char *)io.gtab + off);
                        int32_t ad0 = q - ent.y;
                        ad0 = (active && ad0 >= 0) ? ad0 : -1;
                        done = consume((uint32_t)c + lane * sx, (uint32_t)ent.x, ad0, c, false);
                    }
                    if (done) break;
                }
                n_rows += done ? j + 1 : nb;
                if (done || blast) break;
                // the block's last row, then the next row of the deepest
                // level (sy further), else of a shallower one
                a[MAXM - 1] = ay + (nb - 1) * sy;
                rr[MAXM] = R0 - (nb - 1) * sy * gy;
                plen = plen0 + (nb - 1) * sy;
                xs = 0;
                if ((uint64_t)rr[MAXM] >= (uint64_t)sy * gy) {
                    a[MAXM - 1] += sy;
                    rr[MAXM] -= sy * gy;
                    plen += sy;
                    continue;
                }
                int kk = -1;
#pragma unroll
                for (int k = 0; k + 1 < MAXM; ++k)
                    if (rr[k + 1] >= P.g[k]) kk = k;
                if (kk < 0) break;
#pragma unroll
                for (int k = 0; k < MAXM; ++k) {
                    if (k == kk) {
                        a[k] += 1;
                        rr[k + 1] -= P.g[k];
                    } else if (k > kk) {
                        a[k] = 0;
                        rr[k + 1] = rr[k];
                    }
                }
                plen = 0;
#pragma unroll
                for (int k = 0; k < MAXM; ++k) plen += a[k];
                upper_eq = upper_equal();
            }
        }
        // PACK: rows y = ay + j (j < 64) of the deepest level dl = M - 1, one
        // per lane: its remainder R_j, its lane prefixes x0_j .. xlast_j (none
        // when the row has no element: with PRUNE, when S[M][R_j] = 0) and
        // their exclusive scan, which places the row's prefixes in the block's
        // stream.  Each chunk of 64 stream positions finds every lane's row
        // (the rows that begin inside the chunk, one by one) and solves the
        // lane's x from its remainder alone.
        if constexpr (PACK) {
            const uint32_t dl = M - 1;
            // the lanes' x stride: the common-divisor skip of the last pair
            // (Sec. 3.2.4), D = gcd(A, B) > 1
            const uint32_t sxp = P.cd_sx;
            uint32_t gy = 0;
#pragma unroll
            for (int k = 0; k < MAXM; ++k)
                if (k == (int)dl) gy = P.g[k];
            int pchk = 0; // PRUNE: levels < pchk known to have elements
            while (!done) {
                if constexpr (PRUNE) {
                    // the upper levels must have completions (and the first
                    // row too: skip_empty moves to the first row that has)
                    bool moved = false;
                    if (!skip_empty<MAXM>(P, M, io.S, a, rr, e, end_open, pchk, moved, lane)) break;
                    if (moved) xs = 0;
                }
                uint32_t ay = 0, ey = 0;
                bool ueq = !end_open; // the upper levels equal the end prefix's
                plen = 0;
#pragma unroll
                for (int k = 0; k < MAXM; ++k) {
                    if (k == (int)dl) {
                        ay = a[k];
                        ey = e[k];
                    }
                    if (k < (int)dl) ueq = ueq && a[k] == e[k];
                    plen += a[k];
                }
                const uint32_t R0 = rr[MAXM];
                const uint64_t off = (uint64_t)lane * gy;
                bool in = M > 0 ? off <= R0 : lane == 0;
                if (ueq) in = in && ay + lane <= ey;
                const uint32_t nb = (uint32_t)__builtin_popcountll(__ballot(in));
                const bool end_here = ueq && ay + nb - 1 == ey;
                const uint32_t R = R0 - (uint32_t)off; // meaningful for lanes in
                int32_t x0 = lane == 0 ? xs : 0;
                const int32_t xl_row =
                    (end_here && lane + 1 == nb) ? xe - 1 : (int32_t)fdiv(R, P.div_G2);
                bool has = in && xl_row >= x0;
                if (sxp > 1 && has) {
                    // only x with x G2 = R (mod D) can have an element: none
                    // when e2 does not divide R, else every sxp-th x from
                    // the first at or after x0
                    const uint32_t r2 = fmod32(R, P.div_D);
                    const uint32_t q2 = fdiv(r2, P.div_e2);
                    const uint32_t xst = fmod32(q2 * P.cd_inv2, P.div_sx);
                    x0 += (int32_t)fmod32(xst + sxp - fmod32((uint32_t)x0, P.div_sx), P.div_sx);
                    has = r2 == q2 * P.cd_e2 && xl_row >= x0;
                }
                if constexpr (PRUNE)
                    if (has) has = io.S[(uint64_t)M * P.stride + R] != 0;
                const uint32_t np =
                    has ? (sxp > 1 ? (uint32_t)(xl_row - x0) / sxp : (uint32_t)(xl_row - x0)) + 1u
                        : 0u;
                lane_pref64 += np;
                const uint64_t excl = wave_incl_scan64(np, lane) - np;
                const uint64_t T = readlane64(excl + np, FZK_WAVE - 1);
                const uint32_t exlo = (uint32_t)excl;
                n_rows += nb;
                if constexpr (MODE == FZM_EXISTS) {
                    const uint32_t f = __hip_atomic_load(io.found, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                    if (uni(f)) break;
                }
                for (uint64_t p0 = 0; p0 < T; p0 += FZK_WAVE) {
                    // the row holding position p0 (the last non-empty row
                    // that begins at or before it), then the rows that begin
                    // inside the chunk
                    const uint64_t le = __ballot(np != 0 && excl <= p0);
                    uint32_t jl = (FZK_WAVE - 1) - (uint32_t)__builtin_clzll(le);
                    uint64_t st = __ballot(np != 0 && excl > p0 && excl < p0 + FZK_WAVE);
                    while (st) {
                        const uint32_t j = (uint32_t)__builtin_ctzll(st);
                        st &= st - 1;
                        const uint32_t sj = __builtin_amdgcn_readlane(exlo, j) - (uint32_t)p0;
                        jl = lane >= sj ? j : jl;
                    }
                    const bool active = p0 + lane < T;
                    const uint32_t Rj = (uint32_t)__shfl((int)R, (int)jl, FZK_WAVE);
                    const uint32_t ej = (uint32_t)__shfl((int)exlo, (int)jl, FZK_WAVE);
                    // x = x0_j + sxp (p - excl_j); the lane's remainder Rj - x G2 >= 0
                    const uint32_t k = (uint32_t)p0 + lane - ej;
                    const uint32_t x = sxp > 1 ? (uint32_t)__shfl(x0, (int)jl, FZK_WAVE) + sxp * k
                                               : (jl == 0 ? (uint32_t)xs : 0u) + k;
                    const uint32_t Rc = Rj - x * P.G2;
                    const uint32_t Qv = fdiv(Rc, P.div_B);
                    const uint32_t Pv = Rc - Qv * P.B;
                    const uint32_t ti = active ? Pv + P.B : 0u;
                    const int2 ent = TLDS ? io.ltab[ti] : io.gtab[ti];
                    int32_t ad0 = (int32_t)(Qv - 1) - ent.y;
                    ad0 = (active && ad0 >= 0) ? ad0 : -1;
                    // the row's length offset jl rides on x (plen is row 0's)
                    if (consume(x + jl, (uint32_t)ent.x, ad0, 0, false)) {
                        done = true;
                        break;
                    }
                }
                if (done || (ueq && ay + nb > ey) || M == 0) break;
                // the block's last row, then the next row of the deepest
                // level, else of a shallower one
                uint32_t ylast = ay + nb - 1, rlast = R0 - (nb - 1) * gy;
                xs = 0;
                if (rlast >= gy) {
                    ylast += 1;
                    rlast -= gy;
#pragma unroll
                    for (int k = 0; k < MAXM; ++k)
                        if (k == (int)dl) a[k] = ylast;
#pragma unroll
                    for (int k = 1; k <= MAXM; ++k)
                        if (k > (int)dl) rr[k] = rlast;
                    pchk = (int)dl;
                    continue;
                }
                int kk = -1;
#pragma unroll
                for (int k = 0; k < MAXM; ++k)
                    if (k < (int)dl && rr[k + 1] >= P.g[k]) kk = k;
                if (kk < 0) break;
#pragma unroll
                for (int k = 0; k < MAXM; ++k) {
                    if (k == kk) {
                        a[k] += 1;
                        rr[k + 1] -= P.g[k];
                    } else if (k > kk) {
                        a[k] = 0;
                        rr[k + 1] = rr[k];
                    }
                }
                pchk = kk;
            }
        }
        while (!BLOCKS && !PACK && !done) {
            if (PRUNE && M > 0) {
                bool moved = false;
                if (!skip_empty<MAXM>(P, M, io.S, a, rr, e, end_open, chk, moved, lane)) break;
                if (moved) {
                    xs = 0;
                    plen = 0;
#pragma unroll
                    for (int k = 0; k < MAXM; ++k) plen += a[k];
                    if constexpr (FIXED) upper_eq = upper_equal();
                }
            }
            const uint32_t Rp = rr[MAXM];
            const int32_t xhi = (int32_t)fdiv(Rp, P.div_G2);
            // last row of the slice: the prefix equals the end prefix (the
            // deepest level differs on almost every row, so it goes first)
            bool last = false;
            if constexpr (FIXED) {
                if constexpr (MAXM > 0) last = upper_eq && a[MAXM - 1] == e[MAXM - 1];
                else last = upper_eq;
            } else if (!end_open) {
                last = true;
#pragma unroll
                for (int k = 0; k < MAXM; ++k) last = last && (k >= (int)M || a[k] == e[k]);
            }
            const int32_t xlast = last ? xe - 1 : xhi;
            ++n_rows;
            // the predicate's flag is loaded here and looked at once the row
            // is walked, so that its latency overlaps the row's first loads
            uint32_t found_flag = 0;
            if constexpr (MODE == FZM_EXISTS)
                found_flag =
                    __hip_atomic_load(io.found, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if constexpr (PAIR) {
                // Only the lane prefixes with an element: the pair remainders
                // v = Rp - x G2 (x in [xs, xlast]) that the last pair
                // represents, read from the pair table's chain r = Rp mod G2
                // in descending v (ascending x).  PC[v] counts the chain's
                // representable remainders up to v; PE lists them per chain.
                if (xlast >= xs) {
                    const uint32_t vhi = Rp - (uint32_t)xs * P.G2;
                    const uint32_t vlo = Rp - (uint32_t)xlast * P.G2;
                    const uint32_t r = vhi - fdiv(vhi, P.div_G2) * P.G2;
                    const uint32_t hiE = uni((uint32_t)io.PC[vhi]);
                    const uint32_t loE = vlo >= P.G2 ? uni((uint32_t)io.PC[vlo - P.G2]) : 0u;
                    const uint32_t ro = uni(io.PO[r]);
                    for (uint32_t b = loE; b < hiE; b += FZK_WAVE) {
                        const bool active = b + lane < hiE;
                        const uint32_t kx = b - loE + lane; // position in ascending x
                        const uint32_t v = active ? io.PE[ro + hiE - 1 - kx] : 0u;
                        const uint32_t xl = fdiv(Rp - v, P.div_G2);
                        const uint32_t Qv = fdiv(v, P.div_B);
                        const uint32_t Pv = v - Qv * P.B;
                        const int2 ent = TLDS ? io.ltab[Pv + P.B] : io.gtab[Pv + P.B];
                        int32_t ad0 = (int32_t)(Qv - 1) - ent.y;
                        ad0 = (active && ad0 >= 0) ? ad0 : -1;
                        lane_pref += active ? 1u : 0u;
                        if (consume(xl, (uint32_t)ent.x, ad0, 0, true)) {
                            done = true;
                            break;
                        }
                    }
                }
            } else {
                // Rc = Rp - c G2 = Qc B + Pc, stepped by 64 G2 = c64q B + c64r
                // from chunk to chunk (exact whenever a next chunk exists,
                // since its remainder is >= 0)
                uint32_t Qc, Pc;
                {
                    const uint32_t Rc = Rp - (uint32_t)xs * P.G2;
                    Qc = fdiv(Rc, P.div_B);
                    Pc = Rc - Qc * P.B;
                }
                // The next chunk's table entry is loaded before this chunk is
                // consumed, so that its latency overlaps the consumer's work
                // (a sparse row has many chunks with little to consume).
                // left = xlast - c counts the lanes still to come (no signed
                // overflow near the size limit, where c + 64 would wrap).
                int2 ent;
                if (xs <= xlast) {
                    const uint32_t ti = (int32_t)lane <= xlast - xs ? Pc + lr2 : 0u;
                    ent = TLDS ? io.ltab[ti] : io.gtab[ti];
                }
                uint32_t c = (uint32_t)xs;
                for (int32_t left = xlast - xs; left >= 0; left -= FZK_WAVE, c += FZK_WAVE) {
                    const bool active = (int32_t)lane <= left;
                    const int32_t q2 = (int32_t)(Qc - lq1);
                    uint32_t Pn = Pc - c64r, Qn = Qc - c64q;
                    if ((int32_t)Pn < 0) {
                        Pn += P.B;
                        Qn -= 1;
                    }
                    int2 entn = ent;
                    if (left >= FZK_WAVE) {
                        const uint32_t ti = (int32_t)lane <= left - FZK_WAVE ? Pn + lr2 : 0u;
                        entn = TLDS ? io.ltab[ti] : io.gtab[ti];
                    }
                    // a lane with no element starts at -1, so that the common
                    // decrement stays above -(n + 2 A) > -2^31 for every lane
                    int32_t ad0 = q2 - ent.y;
                    ad0 = (active && ad0 >= 0) ? ad0 : -1;
                    lane_pref += active ? 1u : 0u;
                    if (consume(c + lane, (uint32_t)ent.x, ad0, (int32_t)c, false)) {
                        done = true;
                        break;
                    }
                    ent = entn;
                    Pc = Pn;
                    Qc = Qn;
                }
            }
            if (done || last) break;
            if constexpr (MODE == FZM_EXISTS)
                if (uni(found_flag)) break;
            // next row.  Usually the deepest level grows by one (with a
            // compile-time depth, tested first without the general scan).
            if constexpr (FIXED && MAXM > 0) {
                if (rr[MAXM] >= P.g[MAXM - 1]) {
                    a[MAXM - 1] += 1;
                    rr[MAXM] -= P.g[MAXM - 1];
                    plen += 1;
                    xs = 0;
                    chk = MAXM - 1; // levels above it kept their (non-empty) prefix
                    continue;
                }
            }
            // else the rightmost k < M whose a[k] can grow, deeper coordinates reset
            int kk = -1;
#pragma unroll
            for (int k = 0; k < MAXM; ++k)
                if (k < (int)M && rr[k + 1] >= P.g[k]) kk = k;
            if (kk < 0) break;
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                if (k == kk) {
                    a[k] += 1;
                    rr[k + 1] -= P.g[k];
                } else if (k > kk) {
                    a[k] = 0;
                    rr[k + 1] = rr[k];
                }
            }
            plen = 0;
#pragma unroll
            for (int k = 0; k < MAXM; ++k) plen += a[k];
            xs = 0;
            chk = kk; // levels above kk kept their (non-empty) prefix
            if constexpr (FIXED) upper_eq = upper_equal();
        }
    }
    WalkOut o;
    o.elements = MODE == FZM_STORE ? n_el : wave_sum64(lane_el) + n_trail;
    o.rows = n_rows;
    o.prefixes = wave_sum64(lane_pref + lane_pref64);
    return o;
}

// Single query.  Persistent workgroups of four waves; each wave takes slices
// from an atomic cursor.
// LDS: [residue table, 2B int2, when it fits][per-wave consumer scratch].
// VAR (low three bits): 0 plain, 1 skipping empty subtrees, 2 also walking
// only the pair remainders the last pair represents, 3 the variant walk, 4
// and 5 the packed walk without and with skipping; bit 3 (histograms): a
// 32-bit set of LDS bins per wave beside the workgroup's.
template <int M, int MODE, bool TLDS, int VARH>
__global__ void __launch_bounds__(FZK_WG) fz_enum_kernel(FzPlan P, FzBufs Bf)
{
    constexpr int VAR = VARH & 7;
    constexpr bool H32 = MODE == FZM_HIST && (VARH & 8) != 0;
    extern __shared__ __align__(16) uint32_t lds[];
    constexpr uint32_t NP = M + 1;
    const uint32_t lane = __lane_id();
    const uint32_t wave = threadIdx.x / FZK_WAVE;
    const uint32_t W = uni(Bf.ctl->slices); // cut by fz_slices_kernel

    // TLDS: the residue table is staged in LDS (read with ds_read); else it
    // is read from global memory.  Two instantiations keep each pointer's
    // address space known to the compiler.
    int2 *ltab = (int2 *)lds;
    uint32_t *scratch = lds;
    if constexpr (TLDS) {
        for (uint32_t i = threadIdx.x; i < 2 * P.B; i += blockDim.x) ltab[i] = Bf.restab[i];
        scratch = lds + 2 * (((2 * P.B) + 1) & ~1u); // keep 16-byte alignment
    }
    WalkIO io;
    io.ltab = ltab;
    io.gtab = Bf.restab;
    io.wbins = nullptr;
    io.wbins32 = nullptr;
    io.wbins32l = nullptr;
    io.w32k = 0;
    io.gbins = Bf.hist;
    io.found = &Bf.ctl->found;
    io.out = Bf.out;
    io.S = Bf.S;
    io.PC = Bf.PC;
    io.PE = Bf.PE;
    io.PO = Bf.PO;
    io.TO = Bf.TO;
    io.TT = Bf.TT;
    io.trail_m = P.trail ? Bf.ctl->trail_m : 0;
    // Histogram bins in LDS: one 64-bit set for the workgroup (hist_in_lds
    // 1), or (2) besides it a 32-bit set per wave, which takes the wave's
    // runs and is added into the workgroup's set before it could overflow:
    // every difference entry of a wave's set is bounded by the elements the
    // wave added since its last flush, kept below P.hist32_limit <= 2^31 (a
    // slice's exact element count comes from its ranks).  Private 32-bit sets halve the
    // atomics' LDS traffic and keep the waves off each other's bins.  A wave's
    // set has 2^w32k interleaved copies (bin b, copy c at word b 2^w32k + c;
    // lane l adds to copy l mod 2^w32k): the lanes of a chunk often start
    // their runs in the same few bins, and same-bank atomics are served one
    // lane at a time.
    const uint32_t stride32 = (P.nbins + 2) & ~1u; // nbins + 1 words, even
    const uint32_t w32k = P.hist32_copies;
    if constexpr (MODE == FZM_HIST) {
        if (P.hist_in_lds) { // one set of bins for the workgroup's waves
            io.wbins = (uint64_t *)scratch;
            for (uint32_t i = threadIdx.x; i <= P.nbins; i += blockDim.x) io.wbins[i] = 0;
            if (H32) {
                io.wbins32 = (uint32_t *)(io.wbins + stride32) + ((wave * stride32) << w32k);
                io.wbins32l = io.wbins32 + (lane & ((1u << w32k) - 1));
                io.w32k = w32k;
                for (uint32_t i = lane; i < ((P.nbins + 1) << w32k); i += FZK_WAVE)
                    io.wbins32[i] = 0;
            }
        }
    }
    // a wave adds its 32-bit set (each copy sign-extended) into the
    // workgroup's, then clears it
    auto flush32 = [&]() {
        for (uint32_t i = lane; i <= P.nbins; i += FZK_WAVE) {
            int64_t v = 0;
            for (uint32_t c = 0; c < (1u << w32k); ++c) {
                v += (int32_t)io.wbins32[(i << w32k) + c];
                io.wbins32[(i << w32k) + c] = 0;
            }
            if (v != 0)
                __hip_atomic_fetch_add(&io.wbins[i], (uint64_t)v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };
    uint64_t wave_el = 0; // elements in the wave's 32-bit set
    // store scratch per wave: scan (64 x u64), t0, ad0 and x (64 x u32
    // each), then the staging block of 64 rows x d_user words
    const uint32_t store_words = 5 * FZK_WAVE + FZK_WAVE * P.d_user;
    io.s_incl = (uint64_t *)(scratch + wave * store_words);
    io.s_t0 = (uint32_t *)(io.s_incl + FZK_WAVE);
    io.s_ad0 = io.s_t0 + FZK_WAVE;
    io.s_x = io.s_ad0 + FZK_WAVE;
    io.s_stage = io.s_x + FZK_WAVE;
    __syncthreads();

    // The spine of this loop must stay free of lane-dependent branches: every
    // lane takes part in the cursor atomic (only lane 0 adds 1) and every lane
    // stores the same slice record, so the wave walks each slice as a whole.
    // (a wave whose index is past the slice count has nothing to take: it
    // leaves without touching the cursor)
    const bool idle = blockIdx.x * (FZK_WG / FZK_WAVE) + wave >= W;
    for (; !idle;) {
        const uint32_t old = atomicAdd(&Bf.ctl->cursor, lane == 0 ? 1u : 0u);
        const uint32_t s = __builtin_amdgcn_readlane(old, 0);
        if (s >= W) break;
        if constexpr (MODE == FZM_EXISTS) {
            const uint32_t f =
                __hip_atomic_load(&Bf.ctl->found, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (uni(f)) break;
        }
        const uint64_t t_begin = wall_clock64();
        const uint32_t *b0 = Bf.bounds + (uint64_t)s * NP;
        WalkIO ios = io;
        if constexpr (H32) {
            {
                const uint64_t n_s = Bf.base[s + 1] - Bf.base[s];
                if (wave_el + n_s >= P.hist32_limit) {
                    flush32();
                    wave_el = 0;
                }
                if (n_s >= P.hist32_limit) ios.wbins32 = nullptr; // this slice: 64-bit bins
                else wave_el += n_s;
            }
        }
        // (a slice walked into the workgroup's 64-bit set has a walker of
        // its own, so that the 32-bit one tests nothing per run)
        const WalkOut o =
            (H32 && ios.wbins32 != nullptr)
                ? walk_slice<M, MODE, TLDS, (VAR == 1 || VAR == 2 || VAR == 5), (VAR == 2), true,
                             (VAR == 3), (VAR == 4 || VAR == 5), H32>(P, M, b0, b0 + NP,
                                                                      Bf.base[s], ios, lane)
                : walk_slice<M, MODE, TLDS, (VAR == 1 || VAR == 2 || VAR == 5), (VAR == 2), true,
                             (VAR == 3), (VAR == 4 || VAR == 5), false>(P, M, b0, b0 + NP,
                                                                        Bf.base[s], io, lane);
        {
            FzSliceRec rec;
            rec.elements = o.elements;
            rec.rows = o.rows;
            rec.prefixes = o.prefixes;
            rec.t_begin = t_begin;
            rec.t_end = wall_clock64();
            Bf.recs[s] = rec; // the same value from every lane
        }
    }
    if constexpr (MODE == FZM_HIST) {
        if (P.hist_in_lds) { // every wave has left the loop: the bins are whole
            if constexpr (H32) flush32();
            __syncthreads();
            uint64_t *grow = Bf.hist_rows + (uint64_t)blockIdx.x * P.nbins;
            for (uint32_t i = threadIdx.x; i < P.nbins; i += blockDim.x) grow[i] = io.wbins[i];
        }
    }
}

// The histogram consumer leaves a strided difference array (stride
// |ord - delta|, the change of length between consecutive elements of a
// run); running sums along each residue chain turn it into the histogram.
// Stride 0: the bins already are the histogram.  Whole workgroup.
__device__ void integrate_hist(const FzPlan &P, uint64_t *h, uint64_t *part)
{
    const int32_t step = (int32_t)(P.ord - P.delta);
    const uint32_t mag = step < 0 ? (uint32_t)-step : (uint32_t)step;
    if (mag == 0 || mag >= P.nbins) return;
    chain_scan<false>(h, P.nbins, mag, [&](uint32_t v) { return h[v]; }, part);
}

// Adds the walker workgroups' histogram rows (nwg rows of nbins) into hist,
// zeroed beforehand: thread (bin l, group y) sums rows [y R, (y+1) R) of
// column l, so every row is read once, coalesced, by the whole chip.
__global__ void fz_hist_reduce_kernel(const uint64_t *rows, uint32_t nwg, uint32_t nbins,
                                      uint32_t rows_per_group, uint64_t *hist)
{
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nbins) return;
    const uint32_t b0 = blockIdx.y * rows_per_group;
    const uint32_t b1 = b0 + rows_per_group < nwg ? b0 + rows_per_group : nwg;
    uint64_t h = 0;
    for (uint32_t b = b0; b < b1; ++b) h += rows[(uint64_t)b * nbins + l];
    if (h) atomicAdd((unsigned long long *)&hist[l], (unsigned long long)h);
}

// ---------------------------------------------------------------------------
// Finalize: element / row / prefix totals, the slice self-check (each slice
// must have produced exactly the ranks between its bound and the next), the
// integration of the histogram, and min / max length.
// ---------------------------------------------------------------------------
// Slice totals and the self-check over the whole chip: each wave adds its
// slices' sums to the control block (zeroed by the slice kernel).
__global__ void fz_slice_sums_kernel(FzPlan P, FzBufs Bf)
{
    uint64_t el = 0, rows = 0, pref = 0, bad = 0;
    const uint32_t W = Bf.ctl->slices;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < W;
         s += gridDim.x * blockDim.x) {
        const FzSliceRec r = Bf.recs[s];
        el += r.elements;
        rows += r.rows;
        pref += r.prefixes;
        if (P.mode != FZM_EXISTS && !P.notab && r.elements != Bf.base[s + 1] - Bf.base[s])
            bad = 1;
    }
    for (int o = FZK_WAVE / 2; o > 0; o >>= 1) {
        el += __shfl_xor(el, o);
        rows += __shfl_xor(rows, o);
        pref += __shfl_xor(pref, o);
        bad |= __shfl_xor(bad, o);
    }
    if (__lane_id() == 0) {
        FzCtl *c = Bf.ctl;
        if (el) atomicAdd((unsigned long long *)&c->count, (unsigned long long)el);
        if (rows) atomicAdd((unsigned long long *)&c->rows, (unsigned long long)rows);
        if (pref) atomicAdd((unsigned long long *)&c->prefixes, (unsigned long long)pref);
        if (bad) atomicOr(&c->status, (uint32_t)FZS_MISMATCH);
    }
}

__global__ void __launch_bounds__(1024) fz_finalize_kernel(FzPlan P, FzBufs Bf)
{
    __shared__ uint64_t part[1024];
    const uint32_t tid = threadIdx.x, lane = tid % FZK_WAVE, w = tid / FZK_WAVE;
    const uint32_t nw = blockDim.x / FZK_WAVE;
    uint64_t lo = ~0ull, hi = 0;
    if (P.mode == FZM_HIST) {
        integrate_hist(P, Bf.hist, part);
        for (uint32_t l = tid; l < P.nbins; l += blockDim.x)
            if (Bf.hist[l]) {
                lo = l < lo ? l : lo;
                hi = l > hi ? l : hi;
            }
    }
    for (int o = FZK_WAVE / 2; o > 0; o >>= 1) {
        const uint64_t lo2 = __shfl_xor(lo, o), hi2 = __shfl_xor(hi, o);
        lo = lo2 < lo ? lo2 : lo;
        hi = hi2 > hi ? hi2 : hi;
    }
    __shared__ uint64_t mm[2][1024 / FZK_WAVE];
    if (lane == 0) {
        mm[0][w] = lo;
        mm[1][w] = hi;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t L = ~0ull, H = 0;
        for (uint32_t i = 0; i < nw; ++i) {
            L = mm[0][i] < L ? mm[0][i] : L;
            H = mm[1][i] > H ? mm[1][i] : H;
        }
        FzCtl *c = Bf.ctl;
        c->min_len = L;
        c->max_len = H;
        if (P.notab) c->total = c->count; // no count table: the walk's count
        const uint64_t N = c->total;
        c->written = (c->status & FZS_OVERFLOW) ? 0 : (N < P.max_tuples ? N : P.max_tuples);
    }
}


// ---------------------------------------------------------------------------
// splitWork without tables (Sec. 4, Alg. 4.1, and Remark 4.2's check).  A
// slice is the half-open lexicographic range [a, b) of prefixes (a_1 ..
// a_{d-2}); b may be the end of the set.  The new bound c keeps the prefix
// a_1 .. a_{j-1} at the first level j where a and b differ and splits there
// (Alg. 4.1 splits at that leftmost level; here the value of c_j is not
// a_j - 1 but the one that halves the range's estimated number of elements,
// from the leading term of |Z(R)|, so that repeated halving gives slices of
// similar size), with zeros below.  If no value lies strictly between a_j
// and b_j, c is b's prefix down to level j with zeros below when that is
// still below b, else the split is made inside a's own subtree one level
// deeper, and so on.  Returns false when no c lies strictly inside (a, b)
// (Remark 4.2: the slice is then not split; its second half is empty).
// Ascending walk: a worker keeps [a, c), the new one takes [c, b).
// ---------------------------------------------------------------------------
// Value t in (lo, hi) at level j (generator gj, remainder R before it, k
// coordinates after it) with about as many elements in [lo, t) as in [t, hi):
// the completions of values >= t number about (R - t gj)^k / const.
__device__ uint32_t split_value(uint32_t lo, uint32_t hi, uint32_t R, uint32_t gj, uint32_t k)
{
    const double vlo = pow((double)R - (double)lo * gj, (double)k);
    const double rhi = (double)hi * gj > (double)R ? 0.0 : (double)R - (double)hi * gj;
    const double vhi = pow(rhi, (double)k);
    const double mid = pow(0.5 * (vlo + vhi), 1.0 / k);
    double t = ceil(((double)R - mid) / gj);
    if (!(t > (double)lo)) t = (double)lo + 1;       // (also catches NaN)
    if (t > (double)hi - 1) t = (double)hi - 1;
    return (uint32_t)t;
}

__device__ bool split_bound(const FzPlan &P, const uint32_t *a, const uint32_t *b, uint32_t *c)
{
    const uint32_t K = P.d - 2;
    if (a[0] == FZK_SENTINEL) return false; // [end, end): an empty slice
    const bool b_end = b[0] == FZK_SENTINEL;
    uint32_t j = 0, R = P.n;
    if (!b_end)
        while (j < K && a[j] == b[j]) {
            R -= a[j] * P.g[j];
            ++j;
        }
    if (j == K) return false; // a == b: an empty slice
    // at level j: a_j < b_j (or b is the end: every value up to R / g_j)
    const uint32_t hi = b_end ? R / P.g[j] + 1 : b[j];
    for (uint32_t i = 0; i < K; ++i) c[i] = i < j ? a[i] : 0u;
    if (hi - a[j] >= 2) {
        c[j] = split_value(a[j], hi, R, P.g[j], P.d - 1 - j);
        return true;
    }
    if (!b_end) {
        bool deeper = false;
        for (uint32_t i = j + 1; i < K; ++i) deeper = deeper || b[i] != 0;
        if (deeper) { // (prefix, b_j, 0, ..) lies strictly between a and b
            c[j] = b[j];
            return true;
        }
    }
    // inside a's subtree: the first deeper level with room above a's value
    c[j] = a[j];
    R -= a[j] * P.g[j];
    for (uint32_t i = j + 1; i < K; ++i) {
        const uint32_t hv = R / P.g[i] + 1;
        if (hv - a[i] >= 2) {
            c[i] = split_value(a[i], hv, R, P.g[i], P.d - 1 - i);
            return true;
        }
        c[i] = a[i];
        R -= a[i] * P.g[i];
    }
    return false;
}

// Bound 0 is the first prefix (0, .., 0), bound W the end of the set; the
// control block starts as the slice kernel leaves it.
__global__ void fz_split_init_kernel(FzPlan P, FzBufs Bf)
{
    const uint32_t K = P.d - 2;
    for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) {
        Bf.bounds[i] = 0;
        Bf.bounds[(uint64_t)P.n_slices * K + i] = i == 0 ? FZK_SENTINEL : 0u;
    }
    if (threadIdx.x == 0) {
        FzCtl *c = Bf.ctl;
        c->cursor = 0;
        c->found = 0;
        c->status = 0;
        c->slices = P.n_slices;
        c->total = 0;
        c->count = 0;
        c->rows = 0;
        c->prefixes = 0;
        c->written = 0;
    }
}

__global__ void fz_split_round_kernel(FzPlan P, FzBufs Bf, uint32_t r)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (1u << r)) return;
    uint32_t lo = 0, hi = P.n_slices;
    for (uint32_t bit = r; bit-- > 0;) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if ((k >> bit) & 1u) lo = mid;
        else hi = mid;
    }
    // every slice of the range is empty of records until walked
    if (hi - lo < 2) return;
    const uint32_t mid = lo + (hi - lo) / 2;
    const uint32_t K = P.d - 2;
    uint32_t *c = Bf.bounds + (uint64_t)mid * K;
    if (!split_bound(P, Bf.bounds + (uint64_t)lo * K, Bf.bounds + (uint64_t)hi * K, c))
        for (uint32_t i = 0; i < K; ++i) c[i] = Bf.bounds[(uint64_t)hi * K + i]; // empty
}


// ---------------------------------------------------------------------------
// Trailing-index tables (Sec. 6.1, "dynamic behavior").  The elements of a
// row (a_1 .. a_{d-3}) with remainder R are (a_1 .. a_{d-3}, c) for every c
// in Z(R, (G2, A, B)): a full row with R <= m takes them at once.  The count
// reads |Z(R, (G2, A, B))| from the count table's row M (m = n); the store
// copies them from a table of every Z(x), x < m, ascending, 3 words each,
// with TO[x] = the first triple of Z(x) (the exclusive sum of row M), m - 1
// the largest x whose triples fit in P.trail_cap.
// ---------------------------------------------------------------------------
// TO[0..n+1] by one workgroup (block sums, then each thread's block), and m.
__global__ void __launch_bounds__(1024) fz_trail_scan_kernel(FzPlan P, FzBufs Bf)
{
    __shared__ uint64_t part[1024];
    const uint32_t M = P.d - 3;
    const uint64_t *SM = Bf.S + (uint64_t)M * P.stride;
    const uint64_t len = (uint64_t)P.n + 1;
    const uint64_t per = (len + blockDim.x - 1) / blockDim.x;
    const uint64_t b0 = per * threadIdx.x, b1 = b0 + per < len ? b0 + per : len;
    // saturating sums: the offsets stay non-decreasing, and the table only
    // ever holds the x whose offsets are below the cap
    uint64_t s = 0;
    for (uint64_t v = b0; v < b1; ++v) s = sat_add(s, SM[v]);
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (uint32_t i = 0; i < blockDim.x; ++i) {
            const uint64_t t = part[i];
            part[i] = acc;
            acc = sat_add(acc, t);
        }
    }
    __syncthreads();
    uint64_t acc = part[threadIdx.x];
    for (uint64_t v = b0; v < b1; ++v) {
        Bf.TO[v] = acc;
        acc = sat_add(acc, SM[v]);
    }
    if (b1 == len && b0 < b1) Bf.TO[len] = acc;
    __syncthreads();
    if (threadIdx.x == 0) { // the largest m whose triples fit
        uint64_t lo = 0, hi = len; // TO[lo] fits; find the last x with TO[x + 1] <= cap
        if (Bf.TO[1] > P.trail_cap) {
            Bf.ctl->trail_m = 0; // not even Z(0): no row takes the table
        } else {
            while (hi - lo > 1) {
                const uint64_t mid = (lo + hi) / 2;
                if (Bf.TO[mid + 1] <= P.trail_cap) lo = mid;
                else hi = mid;
            }
            Bf.ctl->trail_m = lo + 1; // Z(x) for every x < trail_m
        }
    }
}

// The triples of Z(x), x < m: a wave per x, lanes over c = a_{d-2}; each
// lane's pair elements run from the first valid a_{d-1}, positions from a
// wave scan of the lanes' counts.
__global__ void fz_trail_fill_kernel(FzPlan P, FzBufs Bf)
{
    const uint64_t m = Bf.ctl->trail_m; // the table holds Z(x), x < m
    const uint32_t lane = __lane_id();
    const uint32_t waves = gridDim.x * (blockDim.x / FZK_WAVE);
    for (uint64_t x = blockIdx.x * (blockDim.x / FZK_WAVE) + threadIdx.x / FZK_WAVE; x < m;
         x += waves) {
        uint64_t pos = Bf.TO[x];
        const uint32_t cmax = (uint32_t)x / P.G2;
        for (uint32_t c0 = 0; c0 <= cmax; c0 += FZK_WAVE) {
            const uint32_t c = c0 + lane;
            uint32_t cnt = 0, t0 = 0, e0 = 0;
            if (c <= cmax) {
                const uint32_t R = (uint32_t)x - c * P.G2;
                if (R % P.D == 0) {
                    t0 = (uint32_t)((uint64_t)((R / P.D) % P.ord) * P.inv % P.ord);
                    if ((uint64_t)P.A * t0 <= R) {
                        e0 = (R - P.A * t0) / P.B;
                        cnt = e0 / P.delta + 1;
                    }
                }
            }
            const uint64_t incl = wave_incl_scan64(cnt, lane);
            const uint64_t tot = readlane64(incl, FZK_WAVE - 1);
            uint32_t *dst = Bf.TT + 3 * (pos + incl - cnt);
            for (uint32_t k = 0; k < cnt; ++k) {
                dst[3 * k] = c;
                dst[3 * k + 1] = t0 + k * P.ord;
                dst[3 * k + 2] = e0 - k * P.delta;
            }
            pos += tot;
        }
    }
}

// ---------------------------------------------------------------------------
// Element of each requested rank (fz_unrank): the slice-bound search carried
// through all d coordinates.  A rank >= |Z| sets FZS_MISMATCH and leaves its
// row untouched.
// ---------------------------------------------------------------------------
__global__ void fz_unrank_kernel(FzPlan P, FzBufs Bf, const uint64_t *ranks, uint64_t nr,
                                 uint32_t *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    const uint64_t N = Bf.S[P.n];
    uint64_t r = ranks[i];
    if (N == ~0ull || r >= N) {
        atomicOr(&Bf.ctl->status, FZS_MISMATCH);
        return;
    }
    uint32_t v = P.n;
    uint32_t *dst = out + i * P.d_user - P.pad;
    for (uint32_t k = 0; k + 1 < P.d; ++k) {
        const uint32_t t = unrank_level(Bf.S + (uint64_t)k * P.stride, v, P.g[k], r);
        if (k >= P.pad) dst[k] = t;
        v -= t * P.g[k];
    }
    dst[P.d - 1] = v / P.B;
}

// ---------------------------------------------------------------------------
// Batches.  One launch per step for all queries: count and work tables of the
// sliced queries (one workgroup each), residue tables, slice bounds (one
// thread per boundary), the walker (persistent, work items taken from one
// cursor across all queries: a wave that finishes a slice of one query takes
// the next item, whatever its query), and a per-query finalize.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) fz_batch_dp_kernel(FzBatchBufs B, const uint32_t *ids)
{
    __shared__ uint64_t part[1024];
    const FzBatchQuery &Q = B.queries[ids[blockIdx.x]];
    const FzPlan P = Q.plan; // P.pair is 0: batches walk without the pair table
    dp_query<false>(P, B.tables + Q.s_off, B.tables + Q.c_off, part, nullptr, nullptr, nullptr);
}

// The same tables one row computation at a time for every query (pass p of a
// query: S rows d-2 .. 0, then C row M from the row work, then C rows M-1 ..
// 0), a row shared by G workgroups: job (q, w, G) takes the chains c = w
// mod G of the row, or the w-th G-th of C row M.  A large query's rows then
// use many compute units instead of one.
__global__ void __launch_bounds__(1024) fz_batch_dp_pass_kernel(FzBatchBufs B, const uint32_t *jobs,
                                                                 uint32_t p)
{
    __shared__ uint64_t part[1024];
    const uint32_t q = jobs[3 * blockIdx.x], w = jobs[3 * blockIdx.x + 1],
                   G = jobs[3 * blockIdx.x + 2];
    const FzBatchQuery &Q = B.queries[q];
    const FzPlan P = Q.plan; // P.pair is 0: batches walk without the pair table
    uint64_t *S = B.tables + Q.s_off, *C = B.tables + Q.c_off;
    const uint32_t d = P.d, M = d - 3;
    if (p + 2 <= d) { // S row k = d - 2 - p
        const uint32_t k = d - 2 - p;
        uint64_t *row = S + (uint64_t)k * P.stride;
        if (k + 1 == d - 1)
            chain_scan<true>(
                row, P.stride, P.g[k],
                [&](uint32_t v) { return (v - fdiv(v, P.div_B) * P.B) == 0 ? 1ull : 0ull; }, part,
                w, G);
        else {
            const uint64_t *nxt = S + (uint64_t)(k + 1) * P.stride;
            chain_scan<true>(row, P.stride, P.g[k], [&](uint32_t v) { return nxt[v]; }, part, w, G);
        }
    } else if (p + 1 == d) { // C row M: the work of a row of each remainder
        uint64_t *CM = C + (uint64_t)M * P.stride;
        const uint64_t *SM = S + (uint64_t)M * P.stride;
        const uint32_t per = (P.stride + G - 1) / G;
        const uint32_t v0 = w * per, v1 = min(P.stride, v0 + per);
        for (uint32_t v = v0 + threadIdx.x; v < v1; v += blockDim.x)
            CM[v] = row_work(P, SM, v, fdiv(v, P.div_G2) + 1, nullptr);
    } else { // C row k = M - 1 - (p - d)
        const uint32_t k = M - 1 - (p - d);
        uint64_t *row = C + (uint64_t)k * P.stride;
        const uint64_t *nxt = C + (uint64_t)(k + 1) * P.stride;
        chain_scan<true>(row, P.stride, P.g[k], [&](uint32_t v) { return nxt[v]; }, part, w, G);
    }
}

// Total modelled work C[0][n] and element count S[0][n] of each query with
// tables, for the host to size its slice count and its bins.
__global__ void fz_batch_totals_kernel(FzBatchBufs B, const uint32_t *ids, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const FzBatchQuery &Q = B.queries[ids[i]];
    B.totals[2 * i] = B.tables[Q.c_off + Q.plan.n];
    B.totals[2 * i + 1] = B.tables[Q.s_off + Q.plan.n];
}

__global__ void fz_batch_restab_kernel(FzBatchBufs B)
{
    const FzBatchQuery &Q = B.queries[blockIdx.x];
    const FzPlan P = Q.plan;
    if (P.d == 0) return; // rejected query
    for (uint32_t i = threadIdx.x; i < 2 * P.B; i += blockDim.x)
        B.restabs[Q.tab_off + i] = restab_entry(P, i);
}

// One thread per boundary job.  Queries that are not sliced have one slice,
// from the prefix (0,...,0) to the end of the set.
__global__ void fz_batch_slices_kernel(FzBatchBufs B)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) *B.cursor = 0;
    if (t >= B.n_bjobs) return;
    const FzBatchJob job = B.bjobs[t];
    const FzBatchQuery &Q = B.queries[job.q];
    const FzPlan P = Q.plan;
    const uint32_t bi = Q.bound_off + job.j;
    uint32_t *out = B.bounds + (uint64_t)bi * B.bstride;
    if (!Q.sliced) {
        if (job.j == 0) {
            for (uint32_t k = 0; k + 2 < P.d; ++k) out[k] = 0;
            B.base[bi] = 0;
        } else {
            out[0] = FZK_SENTINEL;
            B.base[bi] = ~0ull;
        }
        return;
    }
    const uint64_t *S = B.tables + Q.s_off;
    const uint64_t *C = B.tables + Q.c_off;
    if (job.j == 0) {
        const uint64_t N = S[P.n];
        B.res[job.q].total = N;
        if (N == ~0ull || C[P.n] == ~0ull) B.res[job.q].status = FZS_OVERFLOW;
        else if (P.mode == FZM_STORE && N > Q.max_total) B.res[job.q].status = FZS_TOOBIG;
    }
    B.base[bi] = slice_bound(P, S, C, Q.n_slices, job.j, out, nullptr); // no pair table
}

// integrate_hist for one wavefront (no workgroup barrier): lane l takes
// chain l % s and band l / s of it when s < 64, else whole chains.
__device__ void wave_integrate(uint64_t *h, uint32_t nb, uint32_t s, uint32_t lane)
{
    if (s == 0 || s >= nb) return;
    if (s >= FZK_WAVE) {
        for (uint32_t c = lane; c < s; c += FZK_WAVE) {
            uint64_t acc = 0;
            for (uint32_t v = c; v < nb; v += s) {
                acc += h[v];
                h[v] = acc;
            }
        }
        return;
    }
    const uint32_t bands = FZK_WAVE / s;
    const uint32_t rows = (nb + s - 1) / s;
    const uint32_t per = (rows + bands - 1) / bands;
    const uint32_t c = lane % s, b = lane / s;
    const uint32_t k0 = b < bands ? b * per : rows;
    const uint32_t k1 = b < bands ? min(rows, k0 + per) : rows;
    uint64_t sum = 0;
    for (uint32_t k = k0; k < k1; k += 8) {
        uint64_t x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t v = (uint64_t)(k + j) * s + c;
            x[j] = (k + j < k1 && v < nb) ? h[v] : 0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) sum += x[j];
    }
    uint64_t carry = 0;
    for (uint32_t bb = 0; bb < bands; ++bb) {
        const uint64_t x = __shfl(sum, (int)(bb * s + c));
        if (bb < b) carry += x;
    }
    for (uint32_t k = k0; k < k1; k += 8) {
        uint64_t x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t v = (uint64_t)(k + j) * s + c;
            x[j] = (k + j < k1 && v < nb) ? h[v] : 0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t v = (uint64_t)(k + j) * s + c;
            carry += x[j];
            if (k + j < k1 && v < nb) h[v] = carry;
        }
    }
}

// The last step of a batch query, by the wave that completed its last item:
// the histogram's integration and min / max length, rows written, and the
// host-visible copy with its flag.
__device__ void finish_query(const FzBatchBufs &B, uint32_t q, const FzBatchQuery &Q,
                             const FzPlan &P, uint32_t lane)
{
    FzBatchResult &R = B.res[q];
    const uint32_t status = uni(R.status);
    uint64_t lo = ~0ull, hi = 0;
    if (P.mode == FZM_HIST && !(status & (FZS_OVERFLOW | FZS_TOOBIG))) {
        uint64_t *bins = B.bins + Q.bins_off;
        const int32_t step = (int32_t)(P.ord - P.delta);
        wave_integrate(bins, P.nbins, step < 0 ? (uint32_t)-step : (uint32_t)step, lane);
        for (uint32_t l = lane; l < P.nbins; l += FZK_WAVE) {
            const uint64_t h = bins[l];
            if (h) {
                lo = l < lo ? l : lo;
                hi = l > hi ? l : hi;
            }
            if (B.host_bins) B.host_bins[Q.bins_off + l] = h;
        }
        for (int o = FZK_WAVE / 2; o > 0; o >>= 1) {
            const uint64_t lo2 = __shfl_xor(lo, o), hi2 = __shfl_xor(hi, o);
            lo = lo2 < lo ? lo2 : lo;
            hi = hi2 > hi ? hi2 : hi;
        }
    }
    if (lane == 0) {
        const uint64_t count = R.count;
        R.min_len = lo;
        R.max_len = hi;
        R.written = P.mode == FZM_STORE ? count : 0;
        if (B.host_res) {
            FzBatchResult *H = B.host_res + q;
            H->count = count;
            H->total = R.total;
            H->min_len = lo;
            H->max_len = hi;
            H->written = P.mode == FZM_STORE ? count : 0;
            H->found = R.found;
            H->status = R.status;
            H->items_done = R.items_done;
        }
    }
    if (B.host_done) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        if (lane == 0)
            __hip_atomic_store(&B.host_done[q], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

template <int MAXM>
__global__ void __launch_bounds__(FZK_WG)
    fz_batch_enum_kernel(FzBatchBufs B, uint32_t lds_bins, uint32_t max_du)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const uint32_t lane = __lane_id();
    const uint32_t wave = threadIdx.x / FZK_WAVE;
    // per-wave LDS: store scratch (scan, t0, ad0, 64 rows), then the
    // histogram: lds_bins 32-bit bins or half as many 64-bit ones
    const uint32_t store_words = max_du ? 5 * FZK_WAVE + FZK_WAVE * max_du : 0;
    const uint32_t bin_words = lds_bins;
    uint32_t *mine = lds + wave * ((store_words + bin_words + 3) & ~3u);
    WalkIO io;
    io.ltab = nullptr;
    io.s_incl = (uint64_t *)mine;
    io.s_t0 = (uint32_t *)(io.s_incl + FZK_WAVE);
    io.s_ad0 = io.s_t0 + FZK_WAVE;
    io.s_x = io.s_ad0 + FZK_WAVE;
    io.s_stage = io.s_x + FZK_WAVE;
    uint32_t *wb = mine + store_words;

    // uniform spine, as in the single-query walker
    for (;;) {
        const uint32_t old = atomicAdd(B.cursor, lane == 0 ? 1u : 0u);
        const uint32_t it = __builtin_amdgcn_readlane(old, 0);
        if (it >= B.n_items) break;
        const uint64_t t_begin = wall_clock64();
        const uint32_t q = uni(B.items[it].q);
        const uint32_t s = uni(B.items[it].j);
        const FzBatchQuery &Q = B.queries[q];
        const FzPlan P = Q.plan;
        const uint32_t M = uni(P.d) - 3;
        const uint32_t mode = uni(P.mode);
        WalkOut o;
        o.elements = o.rows = o.prefixes = 0;
        // nothing to walk for a refused query, nor for a predicate already
        // satisfied (status and found were set by earlier kernels or waves)
        const uint32_t st0 = uni(__hip_atomic_load(&B.res[q].status, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT));
        bool skip = (st0 & (FZS_OVERFLOW | FZS_TOOBIG)) != 0;
        if (mode == FZM_EXISTS) {
            const uint32_t f =
                __hip_atomic_load(&B.res[q].found, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            skip = skip || uni(f) != 0;
        }
        const uint32_t bi = Q.bound_off + s;
        if (!skip) {
            const uint32_t *b0 = B.bounds + (uint64_t)bi * B.bstride;
            const uint32_t *b1 = b0 + B.bstride;
            const uint64_t base = B.base[bi];
            io.gtab = B.restabs + Q.tab_off;
            io.found = &B.res[q].found;
            io.gbins = B.bins + Q.bins_off;
            io.out = Q.out;
            io.S = B.tables + Q.s_off; // read only when P.prune (set for cut queries)
            io.PC = nullptr;
            io.PE = io.PO = nullptr;
            io.TO = nullptr; // (no trailing tables in a batch)
            io.TT = nullptr;
            io.trail_m = 0;
            io.wbins = nullptr;
            io.wbins32 = nullptr;
            io.wbins32l = nullptr;
            io.w32k = 0;
            const uint32_t lds_hist = mode == FZM_HIST ? uni(P.hist_in_lds) : 0u;
            const uint32_t lds_words = lds_hist == 1 ? 2 * P.nbins : P.nbins;
            if (lds_hist) {
                io.wbins = (uint64_t *)wb;
                io.wbins32 = wb;
                for (uint32_t i = lane; i < lds_words; i += FZK_WAVE) wb[i] = 0;
            }
            const bool prune = uni(P.prune) != 0;
            // Order-free consumers take the packed walk, stores the plain one.
            // (Both walks of a consumer in one kernel would double its
            // registers.)
#define FZ_WALK(MD)                                                                                \
    (prune ? walk_slice<MAXM, MD, false, true, false, false>(P, M, b0, b1, base, io, lane)              \
           : walk_slice<MAXM, MD, false, false, false, false>(P, M, b0, b1, base, io, lane))
#define FZ_PACKED(MD)                                                                              \
    (prune ? walk_slice<MAXM, MD, false, true, false, false, false, true>(P, M, b0, b1, base, io,   \
                                                                          lane)                    \
           : walk_slice<MAXM, MD, false, false, false, false, false, true>(P, M, b0, b1, base, io,  \
                                                                           lane))
            if (mode == FZM_COUNT) o = FZ_PACKED(FZM_COUNT);
            else if (mode == FZM_HIST) o = FZ_PACKED(FZM_HIST);
            else if (mode == FZM_EXISTS) o = FZ_PACKED(FZM_EXISTS);
            else o = FZ_WALK(FZM_STORE);
#undef FZ_PACKED
#undef FZ_WALK
            if (lds_hist == 1) {
                const uint64_t *wb64 = (const uint64_t *)wb;
                for (uint32_t i = lane; i < P.nbins; i += FZK_WAVE) {
                    const uint64_t h = wb64[i];
                    if (h) atomicAdd((unsigned long long *)&io.gbins[i], (unsigned long long)h);
                }
            } else if (lds_hist == 2) {
                for (uint32_t i = lane; i < P.nbins; i += FZK_WAVE) {
                    const uint32_t h = wb[i];
                    if (h)
                        atomicAdd((unsigned long long *)&io.gbins[i],
                                  (unsigned long long)(int64_t)(int32_t)h);
                }
            }
        }
        FzSliceRec rec;
        rec.elements = o.elements;
        rec.rows = o.rows;
        rec.prefixes = o.prefixes;
        rec.t_begin = t_begin;
        rec.t_end = wall_clock64();
        B.recs[it] = rec; // the same value from every lane

        // The item's share of its query, then the item count: the wave that
        // completes the query's last item finishes the query.  Each slice of
        // a cut query must have produced exactly its rank range.
        FzBatchResult &R = B.res[q];
        const bool bad = !skip && Q.sliced && mode != FZM_EXISTS &&
                         o.elements != B.base[bi + 1] - B.base[bi];
        if (lane == 0) {
            if (o.elements) atomicAdd((unsigned long long *)&R.count, o.elements);
            if (bad) atomicOr(&R.status, FZS_MISMATCH);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t old_done = atomicAdd(&R.items_done, lane == 0 ? 1u : 0u);
        const uint32_t done = __builtin_amdgcn_readlane(old_done, 0) + 1;
        if (done == uni(Q.n_slices)) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            finish_query(B, q, Q, P, lane);
        }
    }
}

__global__ void fz_zero_kernel(uint64_t *p, uint64_t count)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// One row of a single query's tables: row[v] = running sum along the chains
// mod gk of the source row (or of g_{d-1} | v).
static void launch_dp_row(const FzPlan &p, const FzBufs &b, bool below_div, const uint64_t *src,
                          uint64_t *row, uint32_t gk, hipStream_t s)
{
    const uint32_t rows = (p.stride - 1) / gk + 1;
    const uint32_t cols = gk < p.stride ? gk : p.stride;
    uint32_t nb = cols >= FZK_DP_UNITS ? 1u : FZK_DP_UNITS / cols;
    nb = nb > 64 ? 64 : nb; // the carry of a block sums at most 63 block sums
    nb = nb > rows ? rows : nb;
    const uint32_t rpb = (rows + nb - 1) / nb;
    const uint32_t units = cols * nb; // <= FZK_DP_UNITS when nb > 1
    const dim3 grid((units + 255) / 256), blk(256);
    if (below_div) {
        if (nb > 1)
            hipLaunchKernelGGL(fz_dp_sums_kernel<true>, grid, blk, 0, s, p, src, gk, cols, nb, rpb, b.dpart);
        hipLaunchKernelGGL(fz_dp_apply_kernel<true>, grid, blk, 0, s, p, src, row, gk, cols, nb, rpb,
                           b.dpart);
    } else {
        if (nb > 1)
            hipLaunchKernelGGL(fz_dp_sums_kernel<false>, grid, blk, 0, s, p, src, gk, cols, nb, rpb, b.dpart);
        hipLaunchKernelGGL(fz_dp_apply_kernel<false>, grid, blk, 0, s, p, src, row, gk, cols, nb, rpb,
                           b.dpart);
    }
}

hipError_t fzk_launch_dp(const FzPlan &p, const FzBufs &b, hipStream_t s)
{
    for (int k = (int)p.d - 2; k >= 0; --k) {
        uint64_t *row = b.S + (uint64_t)k * p.stride;
        const uint64_t *src = b.S + (uint64_t)(k + 1) * p.stride;
        launch_dp_row(p, b, k + 1 == (int)p.d - 1, src, row, p.g[k], s);
    }
    if (p.pair) hipLaunchKernelGGL(fz_pair_kernel, dim3(1), dim3(1024), 0, s, p, b);
    const uint32_t wblocks = (p.n + 1 + 255) / 256;
    hipLaunchKernelGGL(fz_dp_work_kernel, dim3(wblocks < 4096 ? wblocks : 4096), dim3(256), 0, s, p, b);
    const int M = (int)p.d - 3;
    for (int k = M - 1; k >= 0; --k) {
        uint64_t *row = b.C + (uint64_t)k * p.stride;
        const uint64_t *src = b.C + (uint64_t)(k + 1) * p.stride;
        launch_dp_row(p, b, false, src, row, p.g[k], s);
    }
    return hipGetLastError();
}

hipError_t fzk_launch_restab(const FzPlan &p, const FzBufs &b, hipStream_t s)
{
    const uint32_t blocks = (2 * p.B + 255) / 256;
    hipLaunchKernelGGL(fz_restab_kernel, dim3(blocks), dim3(256), 0, s, p, b);
    return hipGetLastError();
}

// Table-free slices: W slices cut from the whole set by repeated
// splitWork (Sec. 4): slice [0, W) is halved, then each half, and so on; a
// thread of round r finds its index range by following the bits of its
// index down from [0, W) and writes the bound in the middle of it, split
// from the bounds at the range's ends.  Rounds run until every range holds
// one slice.
hipError_t fzk_launch_split(const FzPlan &p, const FzBufs &b, hipStream_t s)
{
    hipLaunchKernelGGL(fz_split_init_kernel, dim3(1), dim3(64), 0, s, p, b);
    // slices no wave takes (a predicate that stopped) read as empty
    hipLaunchKernelGGL(fz_zero_kernel, dim3(256), dim3(256), 0, s, (uint64_t *)b.recs,
                       (uint64_t)p.n_slices * (sizeof(FzSliceRec) / 8));
    for (uint32_t r = 0; (1ull << r) < p.n_slices; ++r) {
        const uint32_t ranges = 1u << r;
        hipLaunchKernelGGL(fz_split_round_kernel, dim3((ranges + 255) / 256), dim3(256), 0, s, p, b,
                           r);
    }
    if (p.mode == FZM_HIST)
        hipLaunchKernelGGL(fz_zero_kernel, dim3(256), dim3(256), 0, s, b.hist,
                           (uint64_t)p.nbins + 1); // and the spare bin
    return hipGetLastError();
}

hipError_t fzk_launch_trail(const FzPlan &p, const FzBufs &b, hipStream_t s)
{
    hipLaunchKernelGGL(fz_trail_scan_kernel, dim3(1), dim3(1024), 0, s, p, b);
    if (p.mode == FZM_STORE)
        hipLaunchKernelGGL(fz_trail_fill_kernel, dim3(2048), dim3(256), 0, s, p, b);
    return hipGetLastError();
}

hipError_t fzk_launch_slices(const FzPlan &p, const FzBufs &b, hipStream_t s)
{
    const uint32_t blocks = (p.n_slices + p.host_slices + 1 + 255) / 256;
    hipLaunchKernelGGL(fz_slices_kernel, dim3(blocks), dim3(256), 0, s, p, b);
    if (p.mode == FZM_HIST)
        hipLaunchKernelGGL(fz_zero_kernel, dim3(256), dim3(256), 0, s, b.hist,
                           (uint64_t)p.nbins + 1); // and the spare bin
    return hipGetLastError();
}

size_t fzk_enum_lds_bytes(const FzPlan &p)
{
    const uint32_t waves = FZK_WG / FZK_WAVE;
    size_t bytes = p.restab_in_lds ? (size_t)2 * ((2 * p.B + 1) & ~1u) * sizeof(uint32_t) : 0;
    if (p.mode == FZM_HIST && p.hist_in_lds) bytes += ((size_t)p.nbins + 1) * sizeof(uint64_t);
    if (p.mode == FZM_HIST && p.hist_in_lds == 2) // the 64-bit set padded to even words, then 32-bit sets
        bytes += ((size_t)((p.nbins + 2) & ~1u) - (p.nbins + 1)) * sizeof(uint64_t) +
                 ((size_t)waves * ((p.nbins + 2) & ~1u) << p.hist32_copies) * sizeof(uint32_t);
    if (p.mode == FZM_STORE)
        bytes += (size_t)waves * (5 * FZK_WAVE + FZK_WAVE * p.d_user) * sizeof(uint32_t);
    return bytes;
}

template <int M, bool TLDS, int VAR>
static void launch_enum_mt(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s)
{
    const size_t lds = fzk_enum_lds_bytes(p);
    switch (p.mode) {
    case FZM_COUNT:
        hipLaunchKernelGGL((fz_enum_kernel<M, FZM_COUNT, TLDS, VAR>), dim3(nwg), dim3(FZK_WG), lds,
                           s, p, b);
        break;
    case FZM_HIST:
        if (p.hist_in_lds == 2)
            hipLaunchKernelGGL((fz_enum_kernel<M, FZM_HIST, TLDS, VAR | 8>), dim3(nwg), dim3(FZK_WG),
                               lds, s, p, b);
        else
            hipLaunchKernelGGL((fz_enum_kernel<M, FZM_HIST, TLDS, VAR>), dim3(nwg), dim3(FZK_WG),
                               lds, s, p, b);
        break;
    case FZM_EXISTS:
        hipLaunchKernelGGL((fz_enum_kernel<M, FZM_EXISTS, TLDS, VAR>), dim3(nwg), dim3(FZK_WG), lds,
                           s, p, b);
        break;
    default:
        // (the variant walk counts runs in closed form, and the packed walk
        // does not keep rank order: no store)
        hipLaunchKernelGGL(
            (fz_enum_kernel<M, FZM_STORE, TLDS, VAR == 3 || VAR == 4 ? 0 : VAR == 5 ? 1 : VAR>),
            dim3(nwg), dim3(FZK_WG), lds, s, p, b);
        break;
    }
}

// Skipping empty rows, and the pair table (which implies it), need at least
// one row coordinate (M >= 1).
template <int M>
static hipError_t launch_enum_m(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s)
{
    constexpr int V1 = M > 0 ? 1 : 0, V2 = M > 0 ? 2 : 0, V3 = M > 0 ? 3 : 0;
    constexpr int V4 = M > 0 ? 4 : 0, V5 = M > 0 ? 5 : 0;
    if (M > 0 && p.pack) {
        if (p.prune) {
            if (p.restab_in_lds) launch_enum_mt<M, true, V5>(p, b, nwg, s);
            else launch_enum_mt<M, false, V5>(p, b, nwg, s);
        } else {
            if (p.restab_in_lds) launch_enum_mt<M, true, V4>(p, b, nwg, s);
            else launch_enum_mt<M, false, V4>(p, b, nwg, s);
        }
    } else if (M > 0 && p.cdv) {
        if (p.restab_in_lds) launch_enum_mt<M, true, V3>(p, b, nwg, s);
        else launch_enum_mt<M, false, V3>(p, b, nwg, s);
    } else if (M > 0 && p.pair) {
        if (p.restab_in_lds) launch_enum_mt<M, true, V2>(p, b, nwg, s);
        else launch_enum_mt<M, false, V2>(p, b, nwg, s);
    } else if (M > 0 && p.prune) {
        if (p.restab_in_lds) launch_enum_mt<M, true, V1>(p, b, nwg, s);
        else launch_enum_mt<M, false, V1>(p, b, nwg, s);
    } else {
        if (p.restab_in_lds) launch_enum_mt<M, true, 0>(p, b, nwg, s);
        else launch_enum_mt<M, false, 0>(p, b, nwg, s);
    }
    return hipGetLastError();
}

hipError_t fzk_launch_enum(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s)
{
    switch (p.d - 3) {
    case 0: return launch_enum_m<0>(p, b, nwg, s);
    case 1: return launch_enum_m<1>(p, b, nwg, s);
    case 2: return launch_enum_m<2>(p, b, nwg, s);
    case 3: return launch_enum_m<3>(p, b, nwg, s);
    case 4: return launch_enum_m<4>(p, b, nwg, s);
    case 5: return launch_enum_m<5>(p, b, nwg, s);
    case 6: return launch_enum_m<6>(p, b, nwg, s);
    case 7: return launch_enum_m<7>(p, b, nwg, s);
    case 8: return launch_enum_m<8>(p, b, nwg, s);
    case 9: return launch_enum_m<9>(p, b, nwg, s);
    case 10: return launch_enum_m<10>(p, b, nwg, s);
    case 11: return launch_enum_m<11>(p, b, nwg, s);
    case 12: return launch_enum_m<12>(p, b, nwg, s);
    case 13: return launch_enum_m<13>(p, b, nwg, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t fzk_launch_finalize(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s)
{
    if (p.mode == FZM_HIST && p.hist_in_lds && nwg > 0) {
        constexpr uint32_t kRowsPerGroup = 32;
        const dim3 grid((p.nbins + 255) / 256, (nwg + kRowsPerGroup - 1) / kRowsPerGroup);
        hipLaunchKernelGGL(fz_hist_reduce_kernel, grid, dim3(256), 0, s, b.hist_rows, nwg,
                           p.nbins, kRowsPerGroup, b.hist);
    }
    const uint32_t sblocks = (p.n_slices + 255) / 256;
    hipLaunchKernelGGL(fz_slice_sums_kernel, dim3(sblocks < 256 ? sblocks : 256), dim3(256), 0, s, p, b);
    hipLaunchKernelGGL(fz_finalize_kernel, dim3(1), dim3(1024), 0, s, p, b);
    return hipGetLastError();
}

hipError_t fzk_launch_unrank(const FzPlan &p, const FzBufs &b, const uint64_t *ranks,
                             uint64_t nranks, uint32_t *out, hipStream_t s)
{
    if (nranks == 0) return hipSuccess;
    const uint64_t blocks = (nranks + 255) / 256;
    hipLaunchKernelGGL(fz_unrank_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, p, b, ranks,
                       nranks, out);
    return hipGetLastError();
}

template <int MAXM>
static void launch_batch_enum(const FzBatchBufs &b, uint32_t nwg, uint32_t lds_bins,
                              uint32_t max_du, hipStream_t s)
{
    const uint32_t store_words = max_du ? 5 * FZK_WAVE + FZK_WAVE * max_du : 0;
    const uint32_t bin_words = lds_bins;
    const size_t lds = (size_t)(FZK_WG / FZK_WAVE) * ((store_words + bin_words + 3) & ~3u) * 4;
    hipLaunchKernelGGL((fz_batch_enum_kernel<MAXM>), dim3(nwg), dim3(FZK_WG), lds, s, b,
                       lds_bins, max_du);
}

hipError_t fzk_launch_batch_tables(const FzBatchBufs &b, uint32_t n_tabled,
                                   const uint32_t *tabled_ids, uint32_t n_small,
                                   const uint32_t *small_ids, const uint32_t *pass_jobs,
                                   const uint32_t *pass_off, uint32_t n_pass, hipStream_t s)
{
    hipLaunchKernelGGL(fz_zero_kernel, dim3(64), dim3(256), 0, s, (uint64_t *)b.res,
                       (uint64_t)b.nq * (sizeof(FzBatchResult) / 8));
    if (b.n_bins)
        hipLaunchKernelGGL(fz_zero_kernel, dim3(256), dim3(256), 0, s, b.bins, b.n_bins);
    if (n_tabled) {
        if (n_small) // one workgroup per query, every row in turn
            hipLaunchKernelGGL(fz_batch_dp_kernel, dim3(n_small), dim3(1024), 0, s, b, small_ids);
        for (uint32_t p = 0; p < n_pass; ++p) // pass by pass, rows shared by workgroups
            if (pass_off[p + 1] > pass_off[p])
                hipLaunchKernelGGL(fz_batch_dp_pass_kernel, dim3(pass_off[p + 1] - pass_off[p]),
                                   dim3(1024), 0, s, b, pass_jobs + 3 * (size_t)pass_off[p], p);
        hipLaunchKernelGGL(fz_batch_totals_kernel, dim3((n_tabled + 255) / 256), dim3(256), 0, s,
                           b, tabled_ids, n_tabled);
    }
    hipLaunchKernelGGL(fz_batch_restab_kernel, dim3(b.nq), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t fzk_launch_batch_slices(const FzBatchBufs &b, hipStream_t s)
{
    hipLaunchKernelGGL(fz_batch_slices_kernel, dim3((b.n_bjobs + 255) / 256), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t fzk_launch_batch_walk(const FzBatchBufs &b, uint32_t maxm, uint32_t nwg,
                                 uint32_t lds_bins, uint32_t max_du, hipStream_t s)
{
    if (maxm <= 5) launch_batch_enum<5>(b, nwg, lds_bins, max_du, s);
    else launch_batch_enum<13>(b, nwg, lds_bins, max_du, s);
    return hipGetLastError();
}

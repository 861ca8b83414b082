// Reductions over lattices: the pair observables M, A, B and the row-wise
// spin-spin correlation sums D(r).
//
// M = sum_x sigma_x (magnetisation times L^2, section 3.1), and from the pair
// Hamiltonian of eq. (5): A = sum_x sigma_x (tau_up + tau_right),
// B = sum_x sigma_x tau_x, so that H(sigma, tau) = -(J A + q B).  With bit
// 1 = +1, a product of two spins is +1 exactly when their bits agree, so every
// sum is n - 2 * popcount(xor) over the n sites involved: exact integers.
//
// D(r) = sum_x sigma_(i,j) sigma_(i+r,j): the row-wise analogue of the
// correlations of Table 1.  Each row is staged in LDS as a bit string followed
// by a second copy of itself, so that the row rotated by r is a plain funnel
// shift of two LDS words for every r.
#include "sd_kernels.hpp"

namespace sd {

namespace {

__device__ __forceinline__ void add_obs(int64_t* out3, int64_t pc, int64_t dpair, int64_t dself, int64_t n,
                                        int64_t* red) {
    int64_t v[4] = {pc, dpair, dself, n};
    block_sum_i64<4>(v, red);
    if (threadIdx.x == 0) {
        atomicAdd(reinterpret_cast<unsigned long long*>(out3 + 0), (unsigned long long)(2 * v[0] - v[3]));
        atomicAdd(reinterpret_cast<unsigned long long*>(out3 + 1), (unsigned long long)(2 * v[3] - 2 * v[1]));
        atomicAdd(reinterpret_cast<unsigned long long*>(out3 + 2), (unsigned long long)(v[3] - 2 * v[2]));
    }
}

// Packed layouts (L % 32 == 0): one lane per 32-bit word.
__global__ __launch_bounds__(256) void k_observe_packed(const uint32_t* __restrict__ sigma,
                                                         const uint32_t* __restrict__ tau, Geom G,
                                                         int64_t* __restrict__ out3) {
    __shared__ int64_t red[4 * 4];
    const uint32_t W = G.L / 32u;
    const uint32_t n_words = G.n_sites / 32u;
    int64_t pc = 0, dpair = 0, dself = 0, n = 0;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n_words; u += gridDim.x * blockDim.x) {
        const uint32_t j = fdiv(u, G.div_row);
        const uint32_t w = u - j * W;
        const uint32_t s = sigma[u];
        const uint32_t t = tau[u];
        const uint32_t up = tau[(j == G.L - 1 ? 0 : j + 1) * W + w];
        const uint32_t next = tau[j * W + (w == W - 1 ? 0 : w + 1)];
        const uint32_t right = (t >> 1) | (next << 31);
        pc += __popc(s);
        dpair += __popc(s ^ up) + __popc(s ^ right);
        dself += __popc(s ^ t);
        n += 32;
    }
    add_obs(out3, pc, dpair, dself, n, red);
}

// Bit-string layout (any L % 8 == 0): one lane per 64-bit word, the up and
// right neighbour words as windows of tau.
__global__ __launch_bounds__(256) void k_observe_bits(const uint64_t* __restrict__ sigma,
                                                       const uint64_t* __restrict__ tau, Geom G,
                                                       int64_t* __restrict__ out3) {
    __shared__ int64_t red[4 * 4];
    int64_t pc = 0, dpair = 0, dself = 0, n = 0;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < G.n_groups; g += gridDim.x * blockDim.x) {
        uint64_t t, up, right;
        gather_bits<1>(tau, G.L, G.n_groups, G.div_L, g, t, up, right);
        const uint64_t sg = sigma[g];
        pc += __popcll(sg);
        dpair += __popcll(sg ^ up) + __popcll(sg ^ right);
        dself += __popcll(sg ^ t);
        n += 64;
    }
    add_obs(out3, pc, dpair, dself, n, red);
}

__device__ __forceinline__ uint32_t string_bit(const uint64_t* lat, size_t s) {
    return (uint32_t)(lat[s >> 6] >> (s & 63u)) & 1u;
}

// int8 layout, any L: one lane per site.
__global__ __launch_bounds__(256) void k_observe_i8(const int8_t* __restrict__ sigma, const int8_t* __restrict__ tau,
                                                     Geom G, int64_t* __restrict__ out3) {
    __shared__ int64_t red[4 * 4];
    int64_t pc = 0, dpair = 0, dself = 0, n = 0;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < G.n_sites; s += gridDim.x * blockDim.x) {
        const uint32_t j = fdiv(s, G.div_L);
        const uint32_t i = s - j * G.L;
        const int sx = sigma[s] > 0;
        const int tx = tau[s] > 0;
        const int up = tau[(size_t)(j == G.L - 1 ? 0 : j + 1) * G.L + i] > 0;
        const int right = tau[(size_t)j * G.L + (i == G.L - 1 ? 0 : i + 1)] > 0;
        pc += sx;
        dpair += (sx ^ up) + (sx ^ right);
        dself += sx ^ tx;
        n += 1;
    }
    add_obs(out3, pc, dpair, dself, n, red);
}

// Bits of one row, followed by a second copy, in LDS words (bit p of the
// string is bit p % 32 of word p / 32).
constexpr uint32_t kCorrMaxL = 65535;
constexpr uint32_t kCorrWords = (2 * kCorrMaxL + 64) / 32 + 2;

template <int PACKED>
__device__ __forceinline__ void stage_row(const void* sigma, const Geom& G, uint32_t j, uint32_t* row, uint32_t nw2) {
    if constexpr (PACKED == 2) {
        const uint64_t* s = static_cast<const uint64_t*>(sigma);
        const size_t row0 = (size_t)j * G.L;
        for (uint32_t k = threadIdx.x; k < nw2; k += blockDim.x) {
            uint32_t word = 0;
            uint32_t col = (uint32_t)(((uint64_t)32u * k) % G.L);
            for (int b = 0; b < 32; ++b) {
                word |= string_bit(s, row0 + col) << b;
                if (++col == G.L)
                    col = 0;
            }
            row[k] = word;
        }
    } else if constexpr (PACKED) {
        const uint32_t* s = static_cast<const uint32_t*>(sigma);
        const uint32_t W = G.L / 32u;
        for (uint32_t k = threadIdx.x; k < nw2; k += blockDim.x)
            row[k] = s[(size_t)j * W + (k % W)];
    } else {
        const int8_t* s = static_cast<const int8_t*>(sigma) + (size_t)j * G.L;
        for (uint32_t k = threadIdx.x; k < nw2; k += blockDim.x) {
            uint32_t word = 0;
            uint32_t col = (uint32_t)(((uint64_t)32u * k) % G.L);
            for (int b = 0; b < 32; ++b) {
                word |= (uint32_t)(s[col] > 0) << b;
                if (++col == G.L)
                    col = 0;
            }
            row[k] = word;
        }
    }
}

// out[r] += sum over the block's rows of D_row(r), r = blockIdx.x * blockDim.x + tid.
template <int PACKED>
__global__ __launch_bounds__(256) void k_corr_row(const void* __restrict__ sigma, Geom G, int32_t rmax,
                                                   int64_t* __restrict__ out) {
    __shared__ uint32_t row[kCorrWords];
    const uint32_t L = G.L;
    const uint32_t nwr = (L + 31u) / 32u;                 // words covering one row
    const uint32_t nw2 = (2u * L + 63u) / 32u + 1u;       // words of the doubled string
    const uint32_t last_bits = L - 32u * (nwr - 1u);      // valid bits of the last word
    const uint32_t last_mask = last_bits == 32u ? ~0u : ((1u << last_bits) - 1u);
    const int32_t r = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    int64_t acc = 0;
    for (uint32_t j = blockIdx.y; j < L; j += gridDim.y) {
        __syncthreads();
        stage_row<PACKED>(sigma, G, j, row, nw2);
        __syncthreads();
        if (r <= rmax) {
            uint32_t diff = 0;
            for (uint32_t k = 0; k < nwr; ++k) {
                const uint32_t off = 32u * k + (uint32_t)r;
                const uint32_t q = off >> 5, sh = off & 31u;
                const uint32_t rot = sh ? ((row[q] >> sh) | (row[q + 1] << (32u - sh))) : row[q];
                const uint32_t mask = (k == nwr - 1u) ? last_mask : ~0u;
                diff += __popc((row[k] ^ rot) & mask);
            }
            acc += (int64_t)L - 2 * (int64_t)diff;
        }
    }
    if (r <= rmax)
        atomicAdd(reinterpret_cast<unsigned long long*>(out + r), (unsigned long long)acc);
}

// Rows of whole 64-bit words (the packed string with L % 64 == 0, or int8
// rows whose 64-site groups are 16-byte aligned): workgroup (x, y) takes the
// 64 shifts r = 64 x + lane and the R rows from y R on, staged in LDS as
// W = L / 64 words each; wavefront w sums popcount(row ^ row rotated by r)
// over the W words of its rows w, w + 16, ..., the rotation a funnel shift of
// consecutive words.  r >> 6 = x is uniform in the workgroup, so the LDS reads
// are broadcasts.  The 16 wavefronts' sums are added in LDS and each r gets
// one atomic add into out[r] (zeroed first) per workgroup.  Several
// lattices of one size in one launch: lattice z = blockIdx.z, its sums at
// out + z (rmax + 1).
constexpr uint32_t kCorr64Words = 4096;   // staged words (32 KB)
constexpr uint32_t kCorrWaves = 16;

template <bool INT8>
__global__ __launch_bounds__(1024) void k_corr_row64(CorrLattices cl, uint32_t L, uint32_t R, int32_t rmax,
                                                     int64_t* __restrict__ out) {
    __shared__ uint64_t rows[kCorr64Words];
    __shared__ int64_t part[kCorrWaves][64];
    const void* __restrict__ sigma = cl.p[blockIdx.z];
    out += (size_t)blockIdx.z * ((uint32_t)rmax + 1u);
    const uint32_t W = L / 64u;
    const uint32_t j0 = blockIdx.y * R;
    const uint32_t n = j0 + R < L ? R : L - j0;
    for (uint32_t q = threadIdx.x; q < n * W; q += blockDim.x) {
        if constexpr (INT8)
            rows[q] = load_bits64_i8(static_cast<const int8_t*>(sigma) + (size_t)j0 * L + 64u * q);
        else
            rows[q] = static_cast<const uint64_t*>(sigma)[(size_t)j0 * W + q];
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t s = blockIdx.x;   // r >> 6, at most (L - 1) >> 6 = W - 1
    const uint32_t sh = lane;        // r & 63
    int64_t acc = 0;
    for (uint32_t i = wave; i < n; i += kCorrWaves) {
        const uint64_t* row = rows + i * W;
        uint32_t diff = 0;
        // words s .. W - 1 of the row, then 0 .. s - 1: word w + s (mod W) pairs with word w
#pragma unroll 8
        for (uint32_t w = 0; w < W; ++w) {
            uint32_t q0 = w + s;
            q0 = q0 >= W ? q0 - W : q0;
            const uint32_t q1 = q0 + 1u == W ? 0u : q0 + 1u;
            const uint64_t rot = (row[q0] >> sh) | ((row[q1] << 1) << (63u - sh));
            diff += (uint32_t)__popcll(row[w] ^ rot);
        }
        acc += (int64_t)L - 2 * (int64_t)diff;
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) {
        int64_t t = 0;
#pragma unroll
        for (uint32_t k = 0; k < kCorrWaves; ++k)
            t += part[k][lane];
        const uint32_t r = 64u * blockIdx.x + lane;
        if (r <= (uint32_t)rmax)
            atomicAdd(reinterpret_cast<unsigned long long*>(out + r), (unsigned long long)t);
    }
}

// Diagonal correlation sums (section 3.3, Table 1).  Block (x, y): direction
// d = x / (lmax + 1) (0: partner (i+l, j+l), SW-NE; 1: partner (i+l, j-l),
// NW-SE) and l = x % (lmax + 1), rows j = y, y + gridDim.y, ...; the block's
// count of unequal pairs goes to out[x] as (pairs - 2 * unequal) by one atomic.
// Packed: rows are L / 32 words (L % 32 == 0); the partner row's bits from
// column l on are a funnel shift of two of its words.
template <int PACKED>
__global__ __launch_bounds__(256) void k_corr_diag(const void* __restrict__ sigma, Geom G, int32_t lmax,
                                                    int64_t* __restrict__ out) {
    __shared__ int64_t red[2 * 4];
    const uint32_t L = G.L;
    const uint32_t n_l = (uint32_t)lmax + 1u;
    const uint32_t dir = blockIdx.x / n_l, l = blockIdx.x % n_l;
    int64_t diff = 0, pairs = 0;
    if constexpr (PACKED == 1) {
        const uint32_t* s = static_cast<const uint32_t*>(sigma);
        const uint32_t W = L / 32u;
        const uint32_t sh = l & 31u;
        for (uint32_t j = blockIdx.y; j < L; j += gridDim.y) {
            const uint32_t jp = dir == 0 ? (j + l) % L : (j + L - l) % L;
            const uint32_t* row = s + (size_t)j * W;
            const uint32_t* prow = s + (size_t)jp * W;
            for (uint32_t k = threadIdx.x; k < W; k += blockDim.x) {
                uint32_t q0 = k + (l >> 5);
                q0 = q0 >= W ? q0 - W : q0;
                const uint32_t q1 = q0 + 1u == W ? 0u : q0 + 1u;
                const uint32_t rot = sh ? ((prow[q0] >> sh) | (prow[q1] << (32u - sh))) : prow[q0];
                diff += __popc(row[k] ^ rot);
                pairs += 32;
            }
        }
    } else {
        for (uint32_t j = blockIdx.y; j < L; j += gridDim.y) {
            const uint32_t jp = dir == 0 ? (j + l) % L : (j + L - l) % L;
            for (uint32_t i = threadIdx.x; i < L; i += blockDim.x) {
                const uint32_t ip = (i + l) % L;
                const size_t a = (size_t)j * L + i, b = (size_t)jp * L + ip;
                if constexpr (PACKED == 2) {
                    const uint64_t* s = static_cast<const uint64_t*>(sigma);
                    diff += string_bit(s, a) != string_bit(s, b);
                } else {
                    const int8_t* s = static_cast<const int8_t*>(sigma);
                    diff += (s[a] > 0) != (s[b] > 0);
                }
                pairs += 1;
            }
        }
    }
    int64_t v[2] = {diff, pairs};
    block_sum_i64<2>(v, red);
    if (threadIdx.x == 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(out + blockIdx.x), (unsigned long long)(v[1] - 2 * v[0]));
}

}  // namespace

hipError_t launch_observe(int layout, const void* sigma, const void* tau, const Geom& G, int64_t* out3,
                          hipStream_t st) {
    hipError_t e = launch_fill_i64(out3, 3, 0, st);
    if (e != hipSuccess)
        return e;
    if (layout == kLayBits) {
        uint32_t blocks = (G.n_groups + 255u) / 256u;
        blocks = blocks < kMaxBlocks ? blocks : kMaxBlocks;
        hipLaunchKernelGGL(k_observe_bits, dim3(blocks ? blocks : 1), dim3(256), 0, st,
                           static_cast<const uint64_t*>(sigma), static_cast<const uint64_t*>(tau), G, out3);
    } else if (layout == kLayP64 || layout == kLayP32) {
        uint32_t n_words = G.n_sites / 32u;
        uint32_t blocks = (n_words + 255u) / 256u;
        blocks = blocks < kMaxBlocks ? blocks : kMaxBlocks;
        hipLaunchKernelGGL(k_observe_packed, dim3(blocks ? blocks : 1), dim3(256), 0, st,
                           static_cast<const uint32_t*>(sigma), static_cast<const uint32_t*>(tau), G, out3);
    } else {
        uint32_t blocks = (G.n_sites + 255u) / 256u;
        blocks = blocks < kMaxBlocks ? blocks : kMaxBlocks;
        hipLaunchKernelGGL(k_observe_i8, dim3(blocks ? blocks : 1), dim3(256), 0, st,
                           static_cast<const int8_t*>(sigma), static_cast<const int8_t*>(tau), G, out3);
    }
    return hipGetLastError();
}

hipError_t launch_corr_diag(int layout, const void* sigma, const Geom& G, int32_t lmax, int64_t* out,
                            hipStream_t st) {
    const uint32_t n = 2u * ((uint32_t)lmax + 1u);
    hipError_t e = launch_fill_i64(out, n, 0, st);
    if (e != hipSuccess)
        return e;
    uint32_t row_blocks = kMaxBlocks / n;
    row_blocks = row_blocks < G.L ? row_blocks : G.L;
    row_blocks = row_blocks ? row_blocks : 1u;
    const dim3 grid(n, row_blocks);
    if (layout == kLayBits)
        hipLaunchKernelGGL((k_corr_diag<2>), grid, dim3(256), 0, st, sigma, G, lmax, out);
    else if (layout == kLayP64 || layout == kLayP32)
        hipLaunchKernelGGL((k_corr_diag<1>), grid, dim3(256), 0, st, sigma, G, lmax, out);
    else
        hipLaunchKernelGGL((k_corr_diag<0>), grid, dim3(256), 0, st, sigma, G, lmax, out);
    return hipGetLastError();
}

// Any layout: one lattice, k_corr_row's workgroups over rows and shifts (out
// zeroed by the caller).
static hipError_t launch_corr_row_generic(int layout, const void* sigma, const Geom& G, int32_t rmax, int64_t* out,
                                          hipStream_t st) {
    const uint32_t r_chunks = ((uint32_t)rmax + 256u) / 256u;
    uint32_t row_blocks = kMaxBlocks / r_chunks;
    row_blocks = row_blocks < G.L ? row_blocks : G.L;
    row_blocks = row_blocks ? row_blocks : 1u;
    const dim3 grid(r_chunks, row_blocks);
    if (layout == kLayBits)
        hipLaunchKernelGGL((k_corr_row<2>), grid, dim3(256), 0, st, sigma, G, rmax, out);
    else if (layout == kLayP64 || layout == kLayP32)
        hipLaunchKernelGGL((k_corr_row<1>), grid, dim3(256), 0, st, sigma, G, rmax, out);
    else
        hipLaunchKernelGGL((k_corr_row<0>), grid, dim3(256), 0, st, sigma, G, rmax, out);
    return hipGetLastError();
}

hipError_t launch_corr_row_many(int layout, const void* const* sigma, uint32_t n, const Geom& G, int32_t rmax,
                                int64_t* out, hipStream_t st) {
    if (n < 1 || n > kManyMax)
        return hipErrorInvalidValue;
    hipError_t e = launch_fill_i64(out, (size_t)n * ((size_t)rmax + 1), 0, st);
    if (e != hipSuccess)
        return e;
    if (layout == kLayP64 || layout == kLayI8Row) {
        // 16 rows per workgroup (fewer when 16 rows exceed the staging
        // buffer: W > 256), one 64-shift chunk of r per workgroup column,
        // one lattice per grid layer
        CorrLattices cl{};
        for (uint32_t a = 0; a < n; ++a)
            cl.p[a] = sigma[a];
        const uint32_t W = G.L / 64u;
        const uint32_t R = W <= kCorr64Words / kCorrWaves ? kCorrWaves : kCorr64Words / W;
        const dim3 grid(((uint32_t)rmax + 64u) / 64u, (G.L + R - 1u) / R, n);
        const dim3 block(64u * kCorrWaves);
        if (layout == kLayI8Row)
            hipLaunchKernelGGL((k_corr_row64<true>), grid, block, 0, st, cl, G.L, R, rmax, out);
        else
            hipLaunchKernelGGL((k_corr_row64<false>), grid, block, 0, st, cl, G.L, R, rmax, out);
        return hipGetLastError();
    }
    for (uint32_t a = 0; a < n && e == hipSuccess; ++a)
        e = launch_corr_row_generic(layout, sigma[a], G, rmax, out + (size_t)a * ((size_t)rmax + 1), st);
    return e;
}

hipError_t launch_corr_row(int layout, const void* sigma, const Geom& G, int32_t rmax, int64_t* out,
                           hipStream_t st) {
    return launch_corr_row_many(layout, &sigma, 1u, G, rmax, out, st);
}


}  // namespace sd

// Register/LDS Walsh-Hadamard transform of one sample per wavefront, shared by
// the single-plan compression kernel and the batched kernel.
//
// E = p/64 elements per lane in registers.  The transform is the tensor
// product of 2x2 butterflies over the log2(p) bits of the element index, and
// those commute, so each lane first applies the butterflies of the bits it
// holds in registers; the remaining bits (spread across lanes) are brought
// into registers by transposes through LDS, R bits at a time.
#pragma once

#include "pds_device.hpp"

namespace pds {

// ---------------------------------------------------------------------------
// Bit layouts of the fast path.  Element index bits are split into R register
// bits and 6 lane bits.  Phase 0 is the load layout (bits [0, LV) and
// [LV+6, L) in registers, [LV, LV+6) across lanes).  Phase ph >= 1 brings lane
// bits [LV + (ph-1)R, LV + ph R) into registers (the group), filling any spare
// register bits with the lowest other bits.
// ---------------------------------------------------------------------------
template <int L, int LV>
struct FastLayout {
    static constexpr int R = L - 6;
    static constexpr int kPhases = 1 + (6 + R - 1) / R;

    static constexpr int group_start(int ph) { return LV + (ph - 1) * R; }
    static constexpr int group_size(int ph)
    {
        return (ph == 0) ? R : ((6 - (ph - 1) * R) < R ? (6 - (ph - 1) * R) : R);
    }
    static constexpr bool in_group(int ph, int bit)
    {
        return ph > 0 && bit >= group_start(ph) && bit < group_start(ph) + group_size(ph);
    }
    // element bit carried by register bit k in phase ph
    static constexpr int reg_bit(int ph, int k)
    {
        if (ph == 0) return (k < LV) ? k : k + 6;
        if (k < group_size(ph)) return group_start(ph) + k;
        int need = k - group_size(ph);
        for (int b = 0; b < L; ++b) {
            if (in_group(ph, b)) continue;
            if (need == 0) return b;
            --need;
        }
        return -1;
    }
    static constexpr bool is_reg_bit(int ph, int bit)
    {
        for (int k = 0; k < R; ++k)
            if (reg_bit(ph, k) == bit) return true;
        return false;
    }
    // element bit carried by lane bit k in phase ph
    static constexpr int lane_bit(int ph, int k)
    {
        int need = k;
        for (int b = 0; b < L; ++b) {
            if (is_reg_bit(ph, b)) continue;
            if (need == 0) return b;
            --need;
        }
        return -1;
    }
    static constexpr int reg_part(int ph, int ri)
    {
        int e = 0;
        for (int k = 0; k < R; ++k)
            if ((ri >> k) & 1) e |= 1 << reg_bit(ph, k);
        return e;
    }
    __device__ static int lane_part(int ph, int lane)
    {
        int e = 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) e |= ((lane >> k) & 1) << lane_bit(ph, k);
        return e;
    }
};

template <typename T>
struct VecOf;
template <>
struct VecOf<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <>
struct VecOf<double> {
    using type = double2;
    static constexpr int n = 2;
};

// register bits of the load layout taken from the vector width
template <typename T, int L>
struct FastLV {
    static constexpr int E = (1 << L) / 64;
    static constexpr int value = (VecOf<T>::n < E) ? (VecOf<T>::n == 4 ? 2 : 1) : (E == 4 ? 2 : (E == 2 ? 1 : 0));
};

template <typename T>
__device__ inline T flip_sign(T x, uint32_t neg);
template <>
__device__ inline float flip_sign<float>(float x, uint32_t neg)
{
    return __uint_as_float(__float_as_uint(x) ^ (neg << 31));
}
template <>
__device__ inline double flip_sign<double>(double x, uint32_t neg)
{
    return __longlong_as_double(__double_as_longlong(x) ^ ((unsigned long long)neg << 63));
}

template <typename T, int L>
__device__ inline void load_row(T (&x)[(1 << L) / 64], const T* __restrict__ row, int lane)
{
    constexpr int E = (1 << L) / 64;
    constexpr int V = VecOf<T>::n < E ? VecOf<T>::n : E;
    using Vec = typename VecOf<T>::type;
    if constexpr (V == VecOf<T>::n) {
#pragma unroll
        for (int j = 0; j < E / V; ++j) {
            Vec v = *reinterpret_cast<const Vec*>(row + (j * 64 + lane) * V);
            const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
            for (int q = 0; q < V; ++q) x[j * V + q] = pv[q];
        }
    } else {
#pragma unroll
        for (int j = 0; j < E / V; ++j)
#pragma unroll
            for (int q = 0; q < V; ++q) x[j * V + q] = row[(j * 64 + lane) * V + q];
    }
}

template <int E, typename T>
__device__ inline void butterflies(T (&x)[E], int nbits)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (k >= nbits) break;
#pragma unroll
        for (int ri = 0; ri < E; ++ri) {
            if ((ri >> k) & 1) continue;
            T a = x[ri], b = x[ri | (1 << k)];
            x[ri] = a + b;
            x[ri | (1 << k)] = a - b;
        }
    }
}

// Signs of D for this lane's elements in the load layout (bit ri set = -1),
// from the per-coordinate sign bits negbits (bit j of word j/32).
template <typename T, int L>
__device__ inline uint64_t fast_negmask(const uint32_t* negbits, int lane)
{
    constexpr int E = (1 << L) / 64;
    using Lay = FastLayout<L, FastLV<T, L>::value>;
    uint64_t negmask = 0;
    const int lp = Lay::lane_part(0, lane);
#pragma unroll
    for (int ri = 0; ri < E; ++ri) {
        const int e = lp | Lay::reg_part(0, ri);
        negmask |= (uint64_t)((negbits[e >> 5] >> (e & 31)) & 1u) << ri;
    }
    return negmask;
}

// y = H D x of the row in x (load layout), scaled by 1/sqrt(p) and left in
// buf at padded positions (buf holds lds_pad<T>(p - 1) + 1 elements).  Starts
// and ends with a barrier of the workgroup (one wavefront).
template <typename T, int L>
__device__ inline void fast_transform_to_lds(T (&x)[(1 << L) / 64], uint64_t negmask, T* buf, int lane)
{
    constexpr int E = (1 << L) / 64;
    using Lay = FastLayout<L, FastLV<T, L>::value>;
    constexpr int NPH = Lay::kPhases;
    const T scale = (T)(1.0 / sqrt((double)(1 << L)));
#pragma unroll
    for (int ri = 0; ri < E; ++ri) x[ri] = flip_sign<T>(x[ri], (uint32_t)((negmask >> ri) & 1u));
#pragma unroll
    for (int ph = 0; ph < NPH; ++ph) {
        if (ph > 0) {
            // transpose: current layout out, next layout in.  Lane and register
            // parts of an element index have disjoint bits, so pad(lane | reg) =
            // pad(lane) + pad(reg): one base register plus compile-time offsets
            __syncthreads();
            T* base_old = buf + lds_pad<T>(Lay::lane_part(ph - 1, lane));
#pragma unroll
            for (int ri = 0; ri < E; ++ri) base_old[lds_pad<T>(Lay::reg_part(ph - 1, ri))] = x[ri];
            __syncthreads();
            const T* base_new = buf + lds_pad<T>(Lay::lane_part(ph, lane));
#pragma unroll
            for (int ri = 0; ri < E; ++ri) x[ri] = base_new[lds_pad<T>(Lay::reg_part(ph, ri))];
        }
        butterflies<E, T>(x, Lay::group_size(ph));
    }
    __syncthreads();
    T* base = buf + lds_pad<T>(Lay::lane_part(NPH - 1, lane));
#pragma unroll
    for (int ri = 0; ri < E; ++ri) base[lds_pad<T>(Lay::reg_part(NPH - 1, ri))] = x[ri] * scale;
    __syncthreads();
}

}  // namespace pds

// Double-single (FP32-pair) arithmetic for gfx950.
//
// A double-single number is an unevaluated sum hi + lo of two floats with
// |lo| <= ulp(hi)/2 after normalisation, about 48 significant bits (Sec. 2.4
// of the paper quotes an effective 44 bits for its GPU; gfx950 rounds every
// FP32 add/mul to nearest and its FMA is fused with a single rounding, so the
// error-free transformations below are exact here).
//
//  - two_sum: Knuth's branch-free error-free addition, s + e == a + b exactly.
//  - quick_two_sum: Dekker's Fast2Sum, exact when |a| >= |b| or a == 0.
//  - two_prod: exact product through one fused multiply-add.
//  - ds_add: addition in the style of Bailey's DSFUN90 (the paper's Alg. 1):
//    an error-free sum of the high words, the low words folded into the error
//    term, then renormalisation.
//  - ds_mul: DSFUN90-style product: exact high product plus the two cross
//    terms, renormalised.
//  - Sum2: accumulation of many float terms with an error-free two_sum per
//    term and the rounding errors collected in a float (Ogita, Rump & Oishi,
//    "Accurate sum and dot product", 2005); renormalised once at the end.
//
// The whole library is compiled with -ffp-contract=off, so no a*b+c below is
// fused unless written as fmaf.
#pragma once
#include <hip/hip_runtime.h>

struct dsf {
    float hi, lo;
};

__host__ __device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    float bv = s - a;
    float av = s - bv;
    e = (b - bv) + (a - av);
}

__host__ __device__ __forceinline__ void quick_two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    e = b - (s - a);
}

__device__ __forceinline__ void two_prod(float a, float b, float &p, float &e)
{
    p = a * b;
    e = __builtin_fmaf(a, b, -p);
}

__device__ __forceinline__ dsf ds_from_double(double x)
{
    float h = (float)x;
    float l = (float)(x - (double)h);
    return {h, l};
}

__host__ __device__ __forceinline__ double ds_to_double(dsf a)
{
    return (double)a.hi + (double)a.lo;
}

// Both words of a double-single number in one 64-bit word, bit for bit (a
// conversion to double rounds when the words' bits span more than 53 bits).
__device__ __forceinline__ double ds_pack(dsf a)
{
    const unsigned long long u = ((unsigned long long)__float_as_uint(a.lo) << 32) | __float_as_uint(a.hi);
    return __longlong_as_double((long long)u);
}

__device__ __forceinline__ dsf ds_unpack(double w)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(w);
    return {__uint_as_float((unsigned)u), __uint_as_float((unsigned)(u >> 32))};
}

__device__ __forceinline__ dsf ds_add(dsf a, dsf b)
{
    float s, e;
    two_sum(a.hi, b.hi, s, e);
    e = e + (a.lo + b.lo);
    dsf c;
    quick_two_sum(s, e, c.hi, c.lo);
    return c;
}

__device__ __forceinline__ dsf ds_neg(dsf a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ dsf ds_sub(dsf a, dsf b) { return ds_add(a, ds_neg(b)); }

__device__ __forceinline__ dsf ds_mul(dsf a, dsf b)
{
    float p, e;
    two_prod(a.hi, b.hi, p, e);
    e = __builtin_fmaf(a.hi, b.lo, __builtin_fmaf(a.lo, b.hi, e));
    dsf c;
    quick_two_sum(p, e, c.hi, c.lo);
    return c;
}

// Sum2 accumulator: hi carries the running float sum, err the collected
// rounding errors of every partial sum.
struct sum2f {
    float hi, err;
    __device__ __forceinline__ void init() { hi = 0.0f; err = 0.0f; }
    __device__ __forceinline__ void add(float x)
    {
        float s, e;
        two_sum(hi, x, s, e);
        hi = s;
        err += e;
    }
    // Final renormalisation with a full two_sum (|err| may exceed |hi| after
    // heavy cancellation).
    __device__ __forceinline__ dsf result() const
    {
        dsf r;
        two_sum(hi, err, r.hi, r.lo);
        return r;
    }
};

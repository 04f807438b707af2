// Learned proposal for importance-weighted ABC (not in the paper, whose
// proposal is the prior of eq. 2): a defensive mixture
//   q(theta) = (1 - lambda) q_mix(theta) + lambda prior(theta),
// q_mix an 8-component diagonal Gaussian mixture over the standardised
// parameters t = (theta - tc) / ts (component sds multiplied by `inflate`)
// whose every component is truncated to the prior box dimension by dimension
// (a proper density on the box, drawn by inverse CDF with no redraws); each
// draw carries the importance weight prior(theta) / q(theta). Shared by the
// per-series sampler and the batched persistent kernel, so both draw the same
// theta and weight for the same (seed, domain, series, sample index).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "philox.hpp"

namespace abc {

constexpr int MIX_K = 8, MIX_D = 8, MIX_OUT = MIX_K + 2 * MIX_K * MIX_D;  // 136
constexpr float MIX_LOGSIG_LO = -7.0f, MIX_LOGSIG_HI = 3.0f;

struct ProposalBox {
    float lo[8], hi[8];   // prior box
    float tc[8], ts[8];   // standardisation: centre and sd of the prior
    float lambda;         // defensive prior weight
    float log_inflate;    // log of the factor applied to every component sd
};

// Per-row tables of the truncated mixture: for component k and dimension j
// the standardised box [alpha, beta] = ((a_j - mu)/sigma, (b_j - mu)/sigma)
// of the component, where a_j, b_j are the box edges in standardised units;
// kind 0 (alpha < 0 < beta) keeps Phi(alpha), Phi(beta); kind 1 (alpha >= 0)
// keeps the upper-tail masses Q(alpha), Q(beta); kind 2 (beta <= 0) keeps
// Q(-beta), Q(-alpha), so no mass is formed as a difference of numbers near
// one. logz_k = sum_j log Z_kj (Z = truncated mass); a component with a mass
// below 1e-30 in some dimension is dropped (weight 0); if every component is
// dropped, the proposal is the prior itself (weight 1).
struct MixTable {
    float p1[MIX_K * MIX_D], p2[MIX_K * MIX_D];
    int32_t kind[MIX_K * MIX_D];
    float mu[MIX_K * MIX_D], sig[MIX_K * MIX_D], lsig[MIX_K * MIX_D];
    float logw[MIX_K];   // log of the renormalised component weights (-inf: dropped)
    float cum[MIX_K];    // running sums of the renormalised weights
    float logz[MIX_K];
    int32_t empty;       // every component dropped: the proposal is the prior
};

__device__ __forceinline__ float q_upper(float x) { return 0.5f * erfcf(x * 0.70710678118654752440f); }

// Table entry (k, j) of row o; call for every (k, j), then mix_table_finish.
__device__ inline void mix_table_entry(const float* o, const ProposalBox& p, int k, int j, MixTable& t)
{
    const int e = k * MIX_D + j;
    const float mu = o[MIX_K + k * MIX_D + j];
    const float ls = fminf(fmaxf(o[MIX_K + MIX_K * MIX_D + k * MIX_D + j], MIX_LOGSIG_LO), MIX_LOGSIG_HI) +
                     p.log_inflate;
    const float sg = expf(ls);
    const float a = (p.lo[j] - p.tc[j]) / p.ts[j], b = (p.hi[j] - p.tc[j]) / p.ts[j];
    const float al = (a - mu) / sg, be = (b - mu) / sg;
    if (al >= 0.0f) {         // [alpha, beta] in the upper tail
        t.kind[e] = 1;
        t.p1[e] = q_upper(al);
        t.p2[e] = q_upper(be);
    } else if (be <= 0.0f) {  // in the lower tail: the mirrored interval [-beta, -alpha]
        t.kind[e] = 2;
        t.p1[e] = q_upper(-be);
        t.p2[e] = q_upper(-al);
    } else {                  // straddles the mean: Phi(alpha), Phi(beta)
        t.kind[e] = 0;
        t.p1[e] = q_upper(-al);
        t.p2[e] = 1.0f - q_upper(be);
    }
    t.mu[e] = mu;
    t.sig[e] = sg;
    t.lsig[e] = ls;
}

// Truncated mass of entry e.
__device__ inline float entry_mass(const MixTable& t, int e)
{
    return t.kind[e] == 0 ? t.p2[e] - t.p1[e] : t.p1[e] - t.p2[e];
}

__device__ inline void mix_table_finish(const float* o, MixTable& t)
{
    float lmax = -INFINITY;
    for (int k = 0; k < MIX_K; ++k) lmax = fmaxf(lmax, o[k]);
    float w[MIX_K], tot = 0.0f;
    for (int k = 0; k < MIX_K; ++k) {
        float lz = 0.0f;
        bool drop = false;
        for (int j = 0; j < MIX_D; ++j) {
            const float z = entry_mass(t, k * MIX_D + j);
            drop = drop || !(z >= 1e-30f);
            lz += logf(fmaxf(z, 1e-30f));
        }
        t.logz[k] = lz;
        w[k] = drop ? 0.0f : expf(o[k] - lmax);
        tot += w[k];
    }
    float acc = 0.0f;
    for (int k = 0; k < MIX_K; ++k) {
        acc += w[k];
        t.cum[k] = acc;
        t.logw[k] = w[k] > 0.0f ? logf(w[k] / tot) : -INFINITY;
    }
    t.empty = tot > 0.0f ? 0 : 1;
}

// The whole table of one row in one thread.
__device__ inline void mix_table(const float* o, const ProposalBox& p, MixTable& t)
{
    for (int k = 0; k < MIX_K; ++k)
        for (int j = 0; j < MIX_D; ++j) mix_table_entry(o, p, k, j, t);
    mix_table_finish(o, t);
}

// log q_mix(theta) of the truncated mixture (original units).
__device__ inline float mix_logq_trunc(const MixTable& t, const ProposalBox& p, const float th[8])
{
    float logjac = 0.0f;
    for (int j = 0; j < MIX_D; ++j) logjac += logf(p.ts[j]);
    float L[MIX_K], Lmax = -INFINITY;
    for (int k = 0; k < MIX_K; ++k) {
        float c = t.logw[k] - t.logz[k] - 0.5f * MIX_D * 1.83787706640934548356f;
        for (int j = 0; j < MIX_D; ++j) {
            const int e = k * MIX_D + j;
            const float u = ((th[j] - p.tc[j]) / p.ts[j] - t.mu[e]) / t.sig[e];
            c += -0.5f * u * u - t.lsig[e];
        }
        L[k] = c;
        Lmax = fmaxf(Lmax, c);
    }
    float s = 0.0f;
    for (int k = 0; k < MIX_K; ++k) s += expf(L[k] - Lmax);
    return Lmax + logf(s) - logjac;
}

// One proposal draw for sample i on stream (key, domain, series), day 1:
// block 0 word 0 chooses the prior (u < lambda) or the mixture, word 1 the
// component (inverse CDF of the renormalised weights); blocks 1-2 give eight
// uniforms, used directly (prior) or through the inverse normal CDF of each
// dimension's truncated interval (mixture), so every draw lies in the box
// and no draw is repeated. Writes theta, returns prior / q.
__device__ inline float proposal_draw(const MixTable& t, const ProposalBox& p, Key key, uint64_t i,
                                      uint32_t series, uint32_t domain, float th[8])
{
    const uint4 w0 = stream_words(key, i, series, ctr_word3(1, domain, 0));
    const uint4 w1 = stream_words(key, i, series, ctr_word3(1, domain, 1));
    const uint4 w2 = stream_words(key, i, series, ctr_word3(1, domain, 2));
    const uint32_t ww[8] = {w1.x, w1.y, w1.z, w1.w, w2.x, w2.y, w2.z, w2.w};
    float logvol = 0.0f;
    for (int j = 0; j < 8; ++j) logvol += logf(p.hi[j] - p.lo[j]);
    const float u_sel = (float)(w0.x >> 8) * 0x1p-24f;
    if (t.empty) {  // no component has mass in the box: the proposal is the prior
        for (int j = 0; j < 8; ++j)
            th[j] = fmaf(p.hi[j] - p.lo[j], (float)(ww[j] >> 8) * 0x1p-24f, p.lo[j]);
        return 1.0f;
    }
    if (u_sel < p.lambda) {
        for (int j = 0; j < 8; ++j)
            th[j] = fmaf(p.hi[j] - p.lo[j], (float)(ww[j] >> 8) * 0x1p-24f, p.lo[j]);
    } else {
        const float u_c = (float)(w0.y >> 8) * 0x1p-24f * t.cum[MIX_K - 1];
        int comp = MIX_K - 1;
        for (int c = 0; c < MIX_K; ++c)
            if (u_c < t.cum[c]) {
                comp = c;
                break;
            }
        for (int j = 0; j < 8; ++j) {
            const int e = comp * MIX_D + j;
            const float u = ((float)(ww[j] >> 8) + 0.5f) * 0x1p-24f;  // (0, 1)
            const float p1 = t.p1[e], p2 = t.p2[e];
            float x;
            if (t.kind[e] == 0) {          // Phi(x) = p1 + u (p2 - p1)
                x = -1.41421356237309504880f * erfcinvf(2.0f * fmaf(u, p2 - p1, p1));
            } else {                       // tail: Q(y) = p1 - u (p1 - p2), x = +-y
                const float y = 1.41421356237309504880f * erfcinvf(2.0f * fmaf(-u, p1 - p2, p1));
                x = t.kind[e] == 1 ? y : -y;
            }
            const float tt = fmaf(t.sig[e], x, t.mu[e]);
            th[j] = fminf(fmaxf(fmaf(p.ts[j], tt, p.tc[j]), p.lo[j]), p.hi[j]);
        }
    }
    const float lq_mix = mix_logq_trunc(t, p, th);
    const float lq_prior = -logvol;
    float lq;
    if (p.lambda <= 0.0f) {
        lq = lq_mix;
    } else if (p.lambda >= 1.0f) {
        lq = lq_prior;
    } else {
        const float x = logf(1.0f - p.lambda) + lq_mix, y = logf(p.lambda) + lq_prior;
        const float mx = fmaxf(x, y);
        lq = mx + logf(expf(x - mx) + expf(y - mx));
    }
    return expf(lq_prior - lq);
}

// Standardisation of a prior box, as the network uses it.
__host__ inline void proposal_standardiser(const float lo[8], const float hi[8], float tc[8], float ts[8])
{
    for (int j = 0; j < 8; ++j) {
        tc[j] = 0.5f * (lo[j] + hi[j]);
        ts[j] = (hi[j] - lo[j]) / 3.46410161513775458705f;
    }
}

}  // namespace abc

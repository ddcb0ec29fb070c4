// Rules written on the custom connectivity-update interface (rs_custom.hpp):
// the paper's two worked examples (add_diagonal; remove_random's row part,
// removing the target its host part picked), and DEEP R and the topographic
// rewiring re-expressed as row updates around a host update.  The
// re-expressed rules make the same draws in the same order as the dedicated
// kernels, so they produce the same rows bit for bit.
#include "rs_custom.hpp"

namespace rs {
namespace custom {

__device__ __forceinline__ bool row_bit(const uint32_t* bits, int words, int r, int j) {
  return (bits[(int64_t)r * words + (j >> 5)] >> (j & 31)) & 1u;
}

// add_diagonal: every row adds a synapse onto the target with its own index,
// weight 1 (projections with a connectivity bitfield skip a target already
// connected and record the new one).
struct AddDiagonal {
  static size_t smem_bytes(const ProjDev&) { return 0; }
  __device__ bool active(const RowCtx& c) const { return c.id_pre < c.P.n_post; }
  __device__ void begin(RowCtx&) const {}
  __device__ Visit visit(const RowCtx&, const Syn&) const { return {}; }
  __device__ void removed(const RowCtx&, const Syn&) const {}
  __device__ void add(RowCtx& c, Adder& ad) const {
    const ProjDev& P = c.P;
    if (P.conn && row_bit(P.conn, P.words, c.id_pre, c.id_pre)) return;
    if (ad.add_synapse(c.id_pre, 1.0f) && P.conn)
      P.conn[(int64_t)c.id_pre * P.words + (c.id_pre >> 5)] |= 1u << (c.id_pre & 31);
  }
  __device__ void end(const RowCtx&, int, int) const {}
};

// remove_random, row part: remove the first synapse (slot order) onto the
// target the host part chose for the row, and stop.
struct RemovePost {
  const uint32_t* post_ind;  // [n_pre], from the host update
  static size_t smem_bytes(const ProjDev&) { return 0; }
  __device__ bool active(const RowCtx&) const { return true; }
  __device__ void begin(RowCtx&) const {}
  __device__ Visit visit(const RowCtx& c, const Syn& s) const {
    Visit v;
    v.remove = v.stop = (uint32_t)s.id_post == post_ind[c.id_pre];
    return v;
  }
  __device__ void removed(const RowCtx& c, const Syn& s) const {
    if (c.P.conn) atomicAnd(&c.P.conn[(int64_t)c.id_pre * c.P.words + (s.id_post >> 5)], ~(1u << (s.id_post & 31)));
  }
  __device__ void add(RowCtx&, Adder&) const {}
  __device__ void end(const RowCtx&, int, int) const {}
};

// DEEP R, elimination (Sec. 2.1.2): a synapse whose weight sign disagrees
// with the sign bit of its potential connection is removed and its
// connectivity bit cleared; the row's count goes to the dormant variable.
struct DeeprElim {
  static size_t smem_bytes(const ProjDev&) { return 0; }
  __device__ bool active(const RowCtx&) const { return true; }
  __device__ void begin(RowCtx&) const {}
  __device__ Visit visit(const RowCtx& c, const Syn& s) const {
    const bool neg = row_bit(c.P.sign, c.P.words, c.id_pre, s.id_post);
    Visit v;
    v.remove = (s.w > 0.0f && neg) || (s.w < 0.0f && !neg);
    return v;
  }
  __device__ void removed(const RowCtx& c, const Syn& s) const {
    atomicAnd(&c.P.conn[(int64_t)c.id_pre * c.P.words + (s.id_post >> 5)], ~(1u << (s.id_post & 31)));
  }
  __device__ void add(RowCtx&, Adder&) const {}
  __device__ void end(const RowCtx& c, int removed, int) const { c.P.dormant[c.id_pre] = removed; }
};

// DEEP R, formation: a row adds as many synapses as the host update assigned
// it, each at the first drawn target whose connectivity bit is clear (and
// that is not the row itself in a recurrent projection), weight zero.
struct DeeprForm {
  static size_t smem_bytes(const ProjDev&) { return 0; }
  __device__ bool active(const RowCtx& c) const { return c.P.assigned[c.id_pre] > 0; }
  __device__ void begin(RowCtx&) const {}
  __device__ Visit visit(const RowCtx&, const Syn&) const { return {}; }
  __device__ void removed(const RowCtx&, const Syn&) const {}
  __device__ void add(RowCtx& c, Adder& ad) const {
    const ProjDev& P = c.P;
    const int r = c.id_pre;
    uint32_t* row = P.conn + (int64_t)r * P.words;
    auto free_at = [&](int x) { return !((row[x >> 5] >> (x & 31)) & 1u) && !(P.recurrent && x == r); };
    for (int k = 0; k < P.assigned[r]; ++k) {
      int j = -1;
      for (int t = 0; t < MAX_TRIES && j < 0; ++t) {
        const int x = (int)below(c.rng(TAG_DR_TGT, (uint64_t)k, (uint64_t)t), (uint32_t)P.n_post);
        if (free_at(x)) j = x;
      }
      if (j < 0) {
        const int start = (int)below(c.rng(TAG_DR_TGT, (uint64_t)k, MAX_TRIES), (uint32_t)P.n_post);
        for (int d = 0; d < P.n_post && j < 0; ++d)
          if (free_at((start + d) % P.n_post)) j = (start + d) % P.n_post;
      }
      if (j < 0) break;
      row[j >> 5] |= 1u << (j & 31);
      ad.add_synapse(j, 0.0f);
    }
  }
  __device__ void end(const RowCtx&, int, int) const {}
};

// Topographic rewiring (Sec. 2.1.3): a row that received k attempts from the
// host update sets k candidate targets without replacement in its bitfield
// section, removes candidate synapses with a weight-dependent probability
// (draw keyed by the slot), and forms synapses at the remaining candidates in
// ascending target order with the distance-dependent probability while the
// row has room; every candidate bit is cleared.
struct TopoRule {
  TopoDev t;
  const int* kcount;   // [n_pre], from the host update
  static constexpr int CAND_MAX = 4096;  // candidates per row (attempts per update are at most 4096)
  // LDS: the row's bitfield section, the candidates, their count
  static size_t smem_bytes(const ProjDev& P) { return (size_t)P.words * 4 + (CAND_MAX + 1) * 4; }
  __device__ uint32_t* bits(const RowCtx& c) const { return (uint32_t*)c.smem; }
  __device__ int* cand(const RowCtx& c) const { return (int*)(c.smem + (size_t)c.P.words * 4); }
  __device__ bool active(const RowCtx& c) const { return kcount[c.id_pre] > 0; }
  __device__ void begin(RowCtx& c) const {
    const ProjDev& P = c.P;
    uint32_t* b = bits(c);
    const uint32_t* g = t.bits + (int64_t)c.id_pre * P.words;
    for (int w = c.lane; w < P.words; w += WAVE) b[w] = g[w];
    __syncthreads();
    if (c.lane == 0) {
      const int kr = min(min(kcount[c.id_pre], P.n_post), CAND_MAX);
      int* cd = cand(c);
      int got = 0;
      for (int q = 0; q < kr; ++q) {
        int j = -1;
        for (int tr = 0; tr < MAX_TRIES && j < 0; ++tr) {
          const int x = (int)below(c.rng(TAG_TP_TGT, (uint64_t)q, (uint64_t)tr), (uint32_t)P.n_post);
          if (!((b[x >> 5] >> (x & 31)) & 1u)) j = x;
        }
        if (j < 0) {
          const int start = (int)below(c.rng(TAG_TP_TGT, (uint64_t)q, MAX_TRIES), (uint32_t)P.n_post);
          for (int d = 0; d < P.n_post && j < 0; ++d)
            if (!((b[((start + d) % P.n_post) >> 5] >> (((start + d) % P.n_post) & 31)) & 1u)) j = (start + d) % P.n_post;
        }
        if (j < 0) break;
        b[j >> 5] |= 1u << (j & 31);
        cd[got++] = j;
      }
      cd[CAND_MAX] = got;
    }
  }
  __device__ Visit visit(const RowCtx& c, const Syn& s) const {
    Visit v;
    uint32_t* b = bits(c);
    if ((b[s.id_post >> 5] >> (s.id_post & 31)) & 1u) {
      const uint64_t T = s.w < t.g_theta ? t.T_dep : t.T_pot;
      v.remove = (uint64_t)c.rng(TAG_TP_ELIM, (uint64_t)s.slot) < T;
      atomicAnd(&b[s.id_post >> 5], ~(1u << (s.id_post & 31)));
    }
    return v;
  }
  __device__ void removed(const RowCtx&, const Syn&) const {}
  __device__ void add(RowCtx& c, Adder& ad) const {
    uint32_t* b = bits(c);
    int* cd = cand(c);
    const int kr = cd[CAND_MAX];
    for (int a = 1; a < kr; ++a) {  // ascending target order
      const int x = cd[a];
      int q = a - 1;
      while (q >= 0 && cd[q] > x) { cd[q + 1] = cd[q]; --q; }
      cd[q + 1] = x;
    }
    long long blocked = 0;
    for (int q = 0; q < kr; ++q) {
      const int j = cd[q];
      if (!((b[j >> 5] >> (j & 31)) & 1u)) continue;
      b[j >> 5] &= ~(1u << (j & 31));
      const int dx0 = abs(c.id_pre % t.L - j % t.L), dy0 = abs(c.id_pre / t.L - j / t.L);
      const int dx = min(dx0, t.L - dx0), dy = min(dy0, t.L - dy0);
      if ((uint64_t)c.rng(TAG_TP_FORM, (uint64_t)j) < t.T_d2[dx * dx + dy * dy])
        if (!ad.add_synapse(j, t.g_new)) ++blocked;
    }
    if (blocked) atomicAdd((unsigned long long*)&t.stats[2], (unsigned long long)blocked);
  }
  __device__ void end(const RowCtx&, int, int) const {}
};

}  // namespace custom

void launch_add_diagonal(hipStream_t s, const ProjDev& P, int B, long long* stats) {
  custom::launch_row_update(s, P, custom::AddDiagonal{}, 0, 0, B, stats);
}
void launch_remove_post(hipStream_t s, const ProjDev& P, const uint32_t* post_ind, int B, long long* stats) {
  custom::launch_row_update(s, P, custom::RemovePost{post_ind}, 0, 0, B, stats);
}
void launch_deepr_elim_rule(hipStream_t s, const ProjDev& P, int B, long long* stats) {
  custom::launch_row_update(s, P, custom::DeeprElim{}, 0, 0, B, stats);
}
void launch_deepr_form_rule(hipStream_t s, uint64_t seed, const ProjDev& P, int B, uint64_t step, long long* stats) {
  custom::launch_row_update(s, P, custom::DeeprForm{}, seed, step, B, stats);
}
void launch_topo_rule(hipStream_t s, uint64_t seed, const TopoDev& t, uint64_t step, const int* kcount,
                      long long* stats) {
  custom::launch_row_update(s, t.P, custom::TopoRule{t, kcount}, seed, step, 1, stats);
}

}  // namespace rs

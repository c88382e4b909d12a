// Model object of the DPA-1 library (weights, workspace, stream state) and the
// host helpers shared by the inference entry points and the trainer.  Not part
// of the public ABI (include/dpa1.h, include/dpa1_train.h).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "dpa1.h"
#include "dpa1_internal.h"

// Returns from the enclosing function with a dp_status when a HIP call fails.
#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return dpa1::fail(e_ == hipErrorOutOfMemory ? DP_ERR_OOM : DP_ERR_DEVICE,            \
                        "%s: %s (%s)", #expr, hipGetErrorString(e_), __func__);            \
  } while (0)

namespace dpa1 {

struct Linear {  // one dense layer, FP32, padded
  int fin = 0, fout = 0, ldin = 0, ldout = 0;
  int res = RES_NONE;  // residual rule of the forward layer
  float *Wt = nullptr;  // [ldout][ldin]  (forward operand)
  float *Wb = nullptr;  // [ldin][ldout]  (backward operand)
  float *b = nullptr;   // [ldout]
};

inline int residual_rule(int fin, int fout) {
  if (fout == fin) return RES_IDENT;
  if (fout == 2 * fin) return RES_DOUBLE;
  return RES_NONE;
}

struct Timer {
  bool enabled = false;
  struct Pending {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<int64_t, double>> totals;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void collect() {
    for (auto &p : pending) {
      float ms = 0.f;
      (void)hipEventSynchronize(p.b);
      (void)hipEventElapsedTime(&ms, p.a, p.b);
      auto &t = totals[p.name];
      t.first += 1;
      t.second += ms;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  ~Timer() {
    for (auto &p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};


// Sets the calling thread's error message (dp_last_error) and returns code.
int fail(int code, const char *fmt, ...);

}  // namespace dpa1

struct dp_model {
  // hyper-parameters
  int ntypes = 0, tebd = 0, axis = 0, n_attn = 0, dattn = 0, M = 0, sel = 0;
  int bf16 = 0;  // precision of the matrix-core operands (dp_set_precision)
  std::vector<int> emb, fit;
  double rcut = 0, rcut_smth = 0, shift = 0, ln_eps = 0;
  int device = 0;
  // padded widths
  std::vector<int> lde;  // embedding outputs
  std::vector<int> ldf;  // fitting outputs
  int ldM = 0, ldD = 0;
  // weights
  float *type_table = nullptr;  // [ntypes][ntypes][lde[0]]
  float *ws = nullptr;          // [lde[0]]
  std::vector<dpa1::Linear> embl;     // layers 1..n_emb-1 (index l)
  struct Attn {
    float *Wt_qkv, *Wb_qkv, *b_qkv, *Wt_o, *Wb_o, *b_o, *gamma, *beta;
  };
  std::vector<Attn> attn;
  std::vector<dpa1::Linear> fitl;     // layer 0 uses per-type bias fb0
  float *fb0 = nullptr;         // [ntypes][ldf[0]]
  float *w_out = nullptr;       // [ldf.back()]
  float b_out = 0.f;
  float *ebias = nullptr;       // [ntypes]
  std::vector<void *> weight_allocs;
  // workspace
  void *arena = nullptr;   // topology: per-atom and per-centre buffers
  size_t arena_bytes = 0;
  int cap_nloc = -1, cap_nall = -1, cap_ncell = -1;
  void *parena = nullptr;  // per-pair buffers
  size_t parena_bytes = 0;
  long cap_pairs = -1;     // pair rows parena holds (plus 64 of slack), -1 if not laid out
  int cap_pairs_nloc = -1; // topology capacity the pair arena was laid out with
  long want_pairs = 0;     // pair count of a step that outgrew the arena
  double mem_budget = 0;   // workspace budget in bytes (0: unlimited)
  bool recompute = false;  // attention activations shared across layers, recomputed
  int shared_layer = -1;   // layer whose activations the shared buffers hold
  struct WS {
    double *coords, *out_e, *out_f, *out_v, *out_ae, *vir_part;
    int32_t *types, *types_safe;
    int *atom_cell, *cell_count, *cell_start, *cell_fill, *cell_atoms, *nlist, *nnei, *pair_off;
    float *geom;
    std::vector<float *> h, te;        // embedding outputs / tanh parts
    std::vector<float *> qkv, o, xhat, rstd, G;  // per attention layer (G[a] input of layer a)
    std::vector<float *> lam, fstat;   // per attention layer: scaled logits, (m, 1/Z)
    int *ccount, *clist;               // attention class counts [8] and lists [4][nloc]
    float *T, *dmat, *e;
    std::vector<float *> z, tf;        // fitting outputs / tanh parts
    std::vector<float *> fa, fdz;      // fitting backward a_l and dz_l
    float *dD, *dGa, *dGb, *dY, *dO, *dqkv, *dRt, *gw, *gr, *gs, *g, *astat, *qside;
    float *dA;                         // attention dL/dA per (query, key), layout of lam
    std::vector<float *> du, dh;       // embedding backward
  } w;
  dpa1::DevFlags *flags = nullptr;       // device
  dpa1::DevFlags *flags_host = nullptr;  // pinned
  int *ccount_host = nullptr;            // pinned [8]: class counts of a recent step
  int cls_active = 0;                    // attention classes launched by the last forward
  int cls_small = 0;                     // of those, the ones launched on a small grid
  double *bbox = nullptr;          // device [6]: bounding box for open boundaries
  hipStream_t own = nullptr;
  hipStream_t last = nullptr;
  bool have_step = false;
  int last_nloc = 0;
  struct FwdState {
    const double *coords;  // caller's device coordinates of the last forward
    dpa1::CellGrid grid;
    int nloc, nall;
    bool valid;
  } fwd{};
  dpa1::Timer timer;

  ~dp_model() {
    if (arena) (void)hipFree(arena);
    if (parena) (void)hipFree(parena);
    for (void *p : weight_allocs) (void)hipFree(p);
    if (flags) (void)hipFree(flags);
    if (bbox) (void)hipFree(bbox);
    if (flags_host) (void)hipHostFree(flags_host);
    if (ccount_host) (void)hipHostFree(ccount_host);
    if (own) (void)hipStreamDestroy(own);
  }
};


namespace dpa1 {

// (Re)builds the device weights from a weights-file image (format of the
// seeded-input generator).  With refresh set, the image must have the shapes
// of the loaded model and the existing device arrays are overwritten in place
// (synchronously); nothing is allocated.
int load_weights_image(dp_model *m, const std::vector<char> &buf, bool refresh);

}  // namespace dpa1

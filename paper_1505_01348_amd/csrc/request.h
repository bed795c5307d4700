// Host-side pieces of a device-resident solve that the batched call and the
// server share: the layout of one request's device state, its set-up (dirty
// image, bound, data matrix, initial state: the same launches as a single
// solve on the device loop) and its finish (PWLS rescaling, statistics).
#pragma once

#include <cstddef>

#include "../../include/clsimg.h"
#include "kernels.h"

namespace clsimg {

// Byte offsets inside one request's slice of device memory.
struct ReqLayout {
  size_t El, Em, B0, Bb, E, eps, gam, mf, F, U, st, keys, rs, gpw, dinv, Lw, bytes;
  int nkeys;
  int tiles = 1;  // 16-pixel tiles per wave of the request's multiplier blocks
};

// Layout for P antennas and an nl x nm grid; nkeys argmin keys.
ReqLayout request_layout(int P, int nl, int nm, bool pwls, int nkeys);

// Deferred set-up of a batch: the request's launches become items of the two
// batched set-up launches (request_init_batch, beam_setup_batch).  Only for
// the least-squares cost with the MVDR bound from an R^-1 given, FP32 and
// P <= 48.  shared_tables: every request of the batch has the geometry of the
// context's tables, which its steps then read in place of a copy.  Otherwise
// the request's own tables come from the batched tables launch: its positions
// go to pos_host (staging of the parameter upload, at device address pos_dev).
struct SetupItems {
  ReqInitItem* init;
  BeamSetItem* beam;
  bool shared_tables;
  TableItem* table;
  double* pos_host;
  const double* pos_dev;
};

// Enqueue the set-up of request q on stream st into `slice` (laid out by L)
// and fill its outer-step parameters and multiplier item.  Uses the context's
// shared scratch (tables, Cholesky factors) only inside the stream order.
// rinv: R^-1 of the request already factored and checked (MVDR bound of the
// least-squares cost), or null to factor it here.  defer: fill these items
// instead of launching (see SetupItems).
int request_setup(clsimg_ctx* c, clsimg_request& q, const clsimg_opts* o, char* slice, const ReqLayout& L,
                  OuterParams& op, BeamLamItem& it, hipStream_t st, const float2* rinv = nullptr,
                  const SetupItems* defer = nullptr);

// Status and statistics of a finished request from its final outer state;
// enqueues the PWLS rescaling of sigma.  Returns the request's status.
int request_finish(clsimg_request& q, const clsimg_opts* o, char* slice, const ReqLayout& L, const OuterState& S,
                   hipStream_t st);

// The request can run on the device-resident loop (one workgroup per step).
bool request_on_device(int P);

}  // namespace clsimg

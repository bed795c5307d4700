// Device workspace of a context: buffers grown on demand, and the check every
// entry point makes before its first launch that each buffer its kernels
// write or read exists at the size they assume.  A missing or short buffer
// then comes back as CLSIMG_EWORKSPACE instead of a memory fault.  Host code
// only (no HIP types), so the check itself can be unit-tested on the host.
#ifndef CLSIMG_WORKSPACE_H
#define CLSIMG_WORKSPACE_H

#include <stddef.h>

#include <initializer_list>

#include "../../include/clsimg.h"

namespace clsimg {

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// one requirement: `b` must hold at least `bytes` bytes
struct Need {
  const DevBuf* b;
  size_t bytes;
};

inline int need_all(std::initializer_list<Need> list) {
  for (const Need& n : list)
    if (!n.b || !n.b->ptr || n.b->bytes < n.bytes) return CLSIMG_EWORKSPACE;
  return CLSIMG_OK;
}

}  // namespace clsimg

#endif

// Sanitizer driver for the host side of the C ABI: argument validation,
// size queries and the refusal paths of every entry point, called with
// invalid or oversized arguments so that nothing reaches a device (the
// driver runs where no GPU is present).  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code only; exit code 0 when every
// call returned its documented status.  Test infrastructure only.
#include <stdio.h>
#include <string.h>

#include "styleblit.h"

static int failures = 0;
#define EXPECT(call, want)                                                          \
  do {                                                                              \
    const long long rc_ = (long long)(call);                                        \
    if (rc_ != (long long)(want)) {                                                 \
      fprintf(stderr, "%s:%d: %s gave %lld, expected %lld\n", __FILE__, __LINE__, #call, \
              rc_, (long long)(want));                                              \
      ++failures;                                                                   \
    }                                                                               \
  } while (0)

int main() {
  if (strncmp(sb_version(), "styleblit", 9) != 0) ++failures;
  for (int s = -5; s <= 1; ++s)
    if (!sb_status_string(s)) ++failures;
  // sizes
  EXPECT(sb_jitter_len(1920, 1080, 4, 8) > 0, 1);
  EXPECT(sb_jitter_len(0, 1080, 4, 8), -1);
  EXPECT(sb_jitter_len(8193, 8, 1, 8), -1);
  EXPECT(sb_jitter_len(8, 8, 13, 1), -1);
  EXPECT(sb_jitter_len(8, 8, 2, 3), -1);
  EXPECT(sb_exemplar_texels(512, 512) > 512u * 512u, 1);
  EXPECT(sb_exemplar_texels(0, 5), 0);
  EXPECT(sb_lut_workspace_bytes(0, 512, 512, 8) > 0, 1);
  EXPECT(sb_lut_workspace_bytes(3, 512, 512, 8), 0);
  EXPECT(sb_lut_workspace_bytes(1, 512, 512, 13), 0);
  sb_params p = {4, 8, 32, 3, 1u, SB_JITTER_HASH};
  EXPECT(sb_workspace_bytes(1920, 1080, &p) >= 1920u * 1080u * 4u, 1);
  sb_params bad = p;
  bad.radius = 8;
  EXPECT(sb_workspace_bytes(64, 64, &bad), 0);
  bad = p;
  bad.jitter = 7;
  EXPECT(sb_workspace_bytes(64, 64, &bad), 0);
  EXPECT(sb_workspace_bytes(64, 64, nullptr), 0);
  EXPECT(sb_frame_bytes(1920, 1080) >= 1920u * 1080u * 7u, 1);
  EXPECT(sb_frame_bytes(0, 1), 0);
  EXPECT(sb_batch_max_frames() > 0, 1);
  EXPECT(sb_batch_desc_bytes() > 0, 1);
  EXPECT(sb_noalloc_scratch_bytes(), SB_NOALLOC_SCRATCH_BYTES);

  // refusals before any device work
  char fake[64] = {0};
  sb_style st;
  memset(&st, 0, sizeof st);
  st.rgba = reinterpret_cast<const uint32_t *>(fake);
  st.guide = fake;
  st.lut = reinterpret_cast<const uint32_t *>(fake);
  st.sw = st.sh = 512;
  st.fmt = SB_GUIDE_U8X2;
  st.lut_bits = 8;
  uint8_t *rgb = reinterpret_cast<uint8_t *>(fake);
  uint32_t *chunk = reinterpret_cast<uint32_t *>(fake);
  EXPECT(sb_stylize(&st, fake, 64, 64, nullptr, &p, rgb, chunk, nullptr, nullptr, 0, nullptr),
         SB_EINVAL);                                          // no workspace
  EXPECT(sb_stylize(&st, fake, 64, 64, nullptr, &p, rgb, chunk, nullptr, fake, 16, nullptr),
         SB_ENOMEM);                                          // workspace too small
  EXPECT(sb_stylize(nullptr, fake, 64, 64, nullptr, &p, rgb, chunk, nullptr, fake, 1 << 30,
                    nullptr),
         SB_EINVAL);
  EXPECT(sb_stylize(&st, fake, 64, 64, nullptr, &bad, rgb, chunk, nullptr, fake, 1 << 30,
                    nullptr),
         SB_EINVAL);
  sb_params tab = p;
  tab.jitter = SB_JITTER_TABLE;  // table mode without a table
  EXPECT(sb_stylize(&st, fake, 64, 64, nullptr, &tab, rgb, chunk, nullptr, fake, 1 << 30,
                    nullptr),
         SB_EINVAL);
  sb_tune tn;
  memset(&tn, 0, sizeof tn);
  tn.blend_ppt = 3;  // unsupported choice
  EXPECT(sb_stylize_ex(&st, fake, 64, 64, nullptr, &p, rgb, chunk, nullptr, fake, 1 << 30, &tn,
                       nullptr),
         SB_EINVAL);
  memset(&tn, 0, sizeof tn);
  tn.blend_split = 5;
  EXPECT(sb_stylize_ex(&st, fake, 64, 64, nullptr, &p, rgb, chunk, nullptr, fake, 1 << 30, &tn,
                       nullptr),
         SB_EINVAL);
  EXPECT(sb_stylize_seg(&st, fake, nullptr, 64, 64, nullptr, &p, rgb, chunk, nullptr, fake,
                        1 << 30, nullptr, nullptr),
         SB_EINVAL);                                          // labels missing
  EXPECT(sb_stylize_noalloc(&st, fake, 8192, 8192, nullptr, &p, rgb, chunk, nullptr, nullptr),
         SB_ENOMEM);                                          // beyond the static scratch
  EXPECT(sb_stylize_noalloc(&st, nullptr, 64, 64, nullptr, &p, rgb, chunk, nullptr, nullptr),
         SB_EINVAL);
  sb_style st_bad = st;
  st_bad.lut_bits = 9;  // more bits than an 8-bit guide has
  EXPECT(sb_stylize(&st_bad, fake, 64, 64, nullptr, &p, rgb, chunk, nullptr, fake, 1 << 30,
                    nullptr),
         SB_EINVAL);
  st_bad = st;
  st_bad.weights[0] = 200;  // weight above 127
  EXPECT(sb_stylize(&st_bad, fake, 64, 64, nullptr, &p, rgb, chunk, nullptr, fake, 1 << 30,
                    nullptr),
         SB_EINVAL);

  // batches and the per-frame list
  sb_frame fr[3];
  for (int i = 0; i < 3; ++i) {
    memset(&fr[i], 0, sizeof fr[i]);
    fr[i].style = &st;
    fr[i].tgt_guide = fake;
    fr[i].w = 100 + 37 * i;
    fr[i].h = 60 + 11 * i;
    fr[i].params = p;
    fr[i].out_rgb = rgb;
    fr[i].out_chunk = chunk;
  }
  EXPECT(sb_batch_workspace_bytes(fr, 3) > 0, 1);
  EXPECT(sb_batch_workspace_bytes(fr, 0), 0);
  EXPECT(sb_batch_workspace_bytes(fr, sb_batch_max_frames() + 1), 0);
  EXPECT(sb_batch_run(nullptr, fr, 3, fake, 1 << 30, nullptr), SB_EINVAL);
  EXPECT(sb_stylize_frames(fr, 3, fake, 16, nullptr, nullptr), SB_ENOMEM);
  fr[1].params.radius = 9;
  EXPECT(sb_stylize_frames(fr, 3, fake, 1 << 30, nullptr, nullptr), SB_EINVAL);
  EXPECT(sb_batch_workspace_bytes(fr, 3), 0);
  EXPECT(sb_batch_create(nullptr, fake, 1, nullptr, 0, nullptr, nullptr), SB_EINVAL);
  sb_batch *plan = nullptr;
  EXPECT(sb_batch_create(fake, fake, 1, nullptr, 0, nullptr, &plan), SB_EINVAL);  // capture
  EXPECT(sb_batch_create(fake, fake, 0, nullptr, 17, nullptr, &plan), SB_EINVAL);
  EXPECT(sb_batch_destroy(nullptr), SB_EINVAL);

  // serving: configuration refusals
  sb_serve_config cfg;
  memset(&cfg, 0, sizeof cfg);
  sb_request rq;
  memset(&rq, 0, sizeof rq);
  sb_request_result res;
  EXPECT(sb_serve_run(&cfg, &rq, 1, &res), SB_EINVAL);  // no arena
  cfg.arena = fake;
  cfg.arena_bytes = 1 << 20;
  cfg.slots = 9;  // more slots than supported
  cfg.max_batch = 1;
  cfg.workspace = fake;
  cfg.workspace_bytes_per_slot = 1 << 30;
  cfg.desc_dev = cfg.desc_host = fake;
  EXPECT(sb_serve_run(&cfg, &rq, 1, &res), SB_EINVAL);
  cfg.slots = 2;
  rq.style = &st;
  rq.tgt_guide = fake;
  rq.w = 64;
  rq.h = 64;
  rq.params = bad;  // invalid radius
  EXPECT(sb_serve_run(&cfg, &rq, 1, &res), SB_EINVAL);
  rq.params = p;
  cfg.workspace_bytes_per_slot = 16;  // a request that cannot fit a slot's workspace
  EXPECT(sb_serve_run(&cfg, &rq, 1, &res), SB_ENOMEM);
  // guides of many channels: sizes, tree build and query, frames and serving
  EXPECT(sb_texel_bytes(SB_GUIDE_U8XN, 5), 8);
  EXPECT(sb_texel_bytes(SB_GUIDE_U16XN, 5), 16);
  EXPECT(sb_texel_bytes(SB_GUIDE_U8X3, 3), 0);
  EXPECT(sb_texel_bytes(SB_GUIDE_U8XN, 9), 0);
  const size_t tb = sb_tree_bytes(SB_GUIDE_U16XN, 4, 64, 48);
  const size_t twb = sb_tree_workspace_bytes(SB_GUIDE_U16XN, 4, 64, 48);
  EXPECT(tb > 64u * 48u * 8u, 1);
  EXPECT(twb > 64u * 48u * 8u, 1);
  EXPECT(sb_tree_bytes(SB_GUIDE_U16XN, 4, 0, 48), 0);
  const uint8_t w_bad[8] = {1, 2, 200, 4};
  EXPECT(sb_tree_build(fake, SB_GUIDE_U16XN, 4, 64, 48, w_bad, fake, tb, fake, twb, nullptr),
         SB_EINVAL);
  EXPECT(sb_tree_build(fake, SB_GUIDE_U16XN, 4, 64, 48, nullptr, fake, tb - 1, fake, twb,
                       nullptr),
         SB_ENOMEM);
  EXPECT(sb_tree_build(fake, SB_GUIDE_U16XN, 4, 64, 48, nullptr, fake, tb, fake, twb - 1,
                       nullptr),
         SB_ENOMEM);
  EXPECT(sb_tree_build(fake, SB_GUIDE_U8X2, 2, 64, 48, nullptr, fake, tb, fake, twb, nullptr),
         SB_EINVAL);
  sb_style sst;
  memset(&sst, 0, sizeof sst);
  sst.rgba = reinterpret_cast<const uint32_t *>(fake);
  sst.guide = fake;
  sst.sw = 64;
  sst.sh = 48;
  sst.fmt = SB_GUIDE_U16XN;
  sst.channels = 4;
  sst.tree = fake;
  uint32_t qout = 0;
  EXPECT(sb_tree_query(&sst, fake, -1, &qout, nullptr), SB_EINVAL);
  EXPECT(sb_tree_query(&sst, fake, 0, &qout, nullptr), SB_OK);
  sb_style sst_bad = sst;
  sst_bad.lut_bits = 8;
  EXPECT(sb_stylize(&sst_bad, fake, 64, 64, nullptr, &p, rgb, chunk, nullptr, fake, 1 << 30,
                    nullptr),
         SB_EINVAL);
  sst_bad = sst;
  sst_bad.weights[1] = 128;
  EXPECT(sb_stylize(&sst_bad, fake, 64, 64, nullptr, &p, rgb, chunk, nullptr, fake, 1 << 30,
                    nullptr),
         SB_EINVAL);
  EXPECT(sb_stylize_seg(&sst, fake, reinterpret_cast<const uint8_t *>(fake), 64, 64, nullptr, &p, rgb,
                        chunk, nullptr, fake, 1 << 30, nullptr, nullptr),
         SB_EINVAL);
  sb_style *owned = nullptr;
  EXPECT(sb_style_create_n(nullptr, fake, 64, 48, SB_GUIDE_U8XN, 5, nullptr, nullptr, &owned),
         SB_EINVAL);
  EXPECT(owned == nullptr, 1);
  EXPECT(sb_frame_change(nullptr, nullptr, nullptr, nullptr, 16, nullptr, nullptr, 0, nullptr),
         SB_EINVAL);
  EXPECT(sb_jitter_fill(0, 8, 2, 8, 1, 0, nullptr, nullptr), SB_EINVAL);

  printf("host sanitizer driver: %d failures\n", failures);
  return failures ? 1 : 0;
}

"""FP64 CPU oracle of the VGGT-X memory-efficient aggregator (arXiv 2509.25191, Sec. 3.2),
its patch-embedding front end and the camera global alignment (Sec. 3.3).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls
this package; only the test-suite, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP path: the only thing both
sides share is the seeded input generator in ``synth`` (random draws and
storage-format rounding, no aggregator arithmetic).

The oracle is the plain definition of the aggregator forward: every step in
float64 numpy, exact two-pass softmax, no chunking, no streaming.  The paper
states that its memory optimisations (dropping unused layer outputs, bfloat16,
sequential frame chunks) leave the result unchanged apart from precision
(Sec. 3.2; Sec. 4.3, Tab. 3), so the definition is the reference for every
precision the library offers.

Parity status by function (what pins each one is listed in tests/test_oracle.py):
  layer_norm, gelu, linear, attention, block, aggregate, global_block_rows,
  frame_block_frames: pinned (closed forms, library routines, brute force,
  invariants).
  e4m3_encode / e4m3_decode / quantize_rows / block_exponent: pinned (OCP FP8
  definition, exhaustive code table, torch.float8_e4m3fn conversion of the
  exactly scaled block, binade-edge exponents).
  attention_fp8_emulated: pinned by invariants (constant V gives that row
  exactly; error against the exact attention within the E4M3 bound).
  patchify, frame_tokens, embed (the patch-embedding front end): pinned
  (patch embedding against a float64 Conv2d and a brute-force loop, depth-0
  closed form, frame permutation and scene-first token rules).
  ga (global alignment): pinned (residual against rectified-stereo and
  projected-ray constructions, gradient against torch autograd, Adam against
  torch.optim.Adam, histogram weights against a hand-worked example, the
  median rule against numpy.median, pair selection against a camera ring).
  auc (permutation-equivariant AUC@30): pinned (relative pose against the
  4x4 matrix inverse, angles against scipy rotation vectors and a closed-form
  vector pair, a hand-worked three-camera case, the order sensitivity of the
  conventional form and the order invariance of the both-orders form).
  heads.pack_head_inputs: pinned by an index-by-index loop on a small case.
  Agreement of the whole network with a trained VGGT: parity unpinned (no
  trained weights or worked numeric example exist for this path).
"""
from .aggregator import (  # noqa: F401
    layer_norm, gelu, linear, split_heads, merge_heads, softmax_rows, attention,
    attention_probs, block, aggregate, global_block_rows, frame_block_frames,
    frame_bounds, scene_bounds,
)
from .fp8 import (e4m3_decode, e4m3_encode, quantize_rows, attention_fp8_emulated, block_exponent,  # noqa: F401
                  logit_factor, E4M3_MAX)
from .embed import patchify, frame_tokens, embed  # noqa: F401
from . import ga  # noqa: F401
from . import auc  # noqa: F401
from . import heads  # noqa: F401

"""FP64 CPU oracle for neural texture compression (Vaidyanathan et al., arXiv 2305.17105).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import or call anything in this package.
The HIP library never reaches it, and it shares no code with the HIP library.

Every function is a plain, slow, obviously-correct restatement of the paper's
definitions (section / equation / table named in each docstring), evaluated in
float64.  Where the paper is silent the reading taken is stated in the docstring.

Parity status per function (what pins it, see tests/test_oracle_*.py):
  geometry / level_of_mip ........ Table 1 rows, Table 3/6 byte counts (pinned)
  quantize / dequantize / pack ... hand tables, exhaustive code round trip (pinned)
  noise_hash ..................... published SplitMix64 seed-0 outputs (pinned)
  sample_inputs .................. hand-expanded 8x8 neighbour table, bilinear invariants (pinned)
  pos_enc ........................ closed-form values, period 8, constant last value (pinned)
  mlp_forward .................... selection-matrix wiring test, zero-weight bias test (pinned)
  loss_and_grads ................. torch-CPU float64 autograd + central finite differences (pinned)
  adam_update .................... step-1 closed form, constant-gradient closed form (pinned)
  psnr ........................... Eq. 1 hand examples (pinned)
  MLP outputs / training trajectories on synthetic materials: pinned only through
  the component pins above (the paper prints no decoded values).
"""
from .ntc_oracle import *  # noqa: F401,F403

"""FP64 CPU oracle of the Radar-STDA hot path (arXiv 2307.09063).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the CPU-baseline
leg of the benchmark may import or run anything in this package; the product library and
its Python binding never do, and they share no code with it.

  layers   -- convolution / transposed convolution / depthwise / BN / ReLU / ECA and adjoints
  net      -- the network, its hand-written backward, MSE loss, SGD, the parameter layout
  rdsynth  -- FMCW beat signal, windows, 2-D DFT, dB normalisation, Philox noise, SINR / EVM
  detect   -- CA-CFAR peak detection on restored maps and the fraction of reference peaks found
  optim    -- AdamW with decoupled weight decay and step annealing

Parity unpinned (no figure, code or data of the paper fixes them; they are readings):
the block count and widths, the input/output module contents, the depthwise choice of the
stage-1 3x3 branch, the decoder residual (DeConv4x4-s2), the ECA width and placement, the skip
endpoints, the loss, the CA-CFAR window sizes and edge rules, the AdamW moment coefficients and annealing
period, and the realism of the synthetic
scenes against measured data.
"""
from . import detect, layers, net, optim, rdsynth  # noqa: F401

"""MI355X-native Radar-STDA hot path: HIP kernels behind a C ABI (libstda.so) and a thin
Python binding.  Importing the package loads nothing; `paper_2307_09063_amd.stda` loads the
library and fails loudly if it is missing."""

"""Build ``synth/libsynth.so`` (GPU generator of the synthetic inputs) with hipcc."""

import sys

from .gpu import build

if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

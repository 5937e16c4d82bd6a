"""Learned SpMV selector: the trained cost model shipped with the library,
and the scripts that measure its training set and train it on the GPU.

model.bin   weights + feature standardisation (xab_selector_save format)
collect.py  times every selector class on the generated training / held-out
            matrices (run on the GPU)
train.py    trains the 12-64-64-15 MLP with the library's own kernels and
            scores it by regret against the measured timings
report.json held-out regret of model.bin, of the exhaustive TIME policy
            and of the untuned STABLE default
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "model.bin")
DATA_DIR = os.path.join(HERE, "data")

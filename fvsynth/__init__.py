"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only *draws data*: a diagonal GMM and descriptors sampled from it
(plus uniform outliers), the batch size lists and the serving arrival times, and a
stand-in PCA with raw 130-value descriptors built so that their projection is a GMM
sample (built from the sample; the projection itself is not computed here).
It contains none of the Fisher-vector arithmetic, so the GPU path and the
FP64 oracle can both consume it without sharing any of the method.

The paper's inputs (dense-SIFT descriptors PCA-reduced to ~80 dims, a 256-component
GMM trained on Caltech256 / pubfig; Sec. 3.1 and Sec. 4) are not available, so
these generators stand in for them with the paper's shapes (K=256 components,
D of 64-82, ~10^4 descriptors per 320x240 frame).
"""
from .gen import (  # noqa: F401
    Gmm, gmm, frame, batch_sizes, batch_frames, serving_plan, workload, WORKLOADS,
    array_sha256, Pca, pca, raw_frame, raw_batch, image, images,
)

"""Shared helpers of the GPU parity tests: oracle references (FP64, CPU)
and comparison rules.  Tolerances: FSQ indices bit-exact except for tokens
whose bounded value lies within 1e-3 of a rounding boundary (both codes are
correct there); FP32 reconstruction of identical codes max-abs <= 1e-4."""
import functools

import numpy as np

import synth
from oracle import tokenizer as O

BAND = 1e-3
F32_RECON_TOL = 1e-4


@functools.lru_cache(maxsize=None)
def weights(random_affine=False):
    return synth.make_weights(1, random_affine=random_affine)


@functools.lru_cache(maxsize=None)
def weights64(random_affine=False):
    return {k: v.astype(np.float64) for k, v in weights(random_affine).items()}


@functools.lru_cache(maxsize=None)
def clip(seeds, T, H, W):
    return synth.make_batch(list(seeds), T, H, W)


@functools.lru_cache(maxsize=None)
def oracle_roundtrip(seeds, T, H, W, random_affine=False):
    return O.roundtrip(clip(seeds, T, H, W), weights64(random_affine))


def in_band(b):
    """Per token: any channel's bounded value within BAND of a rounding boundary."""
    return (O.fsq_boundary_distance(b) < BAND).any(axis=-1)


def idx_agreement(idx_gpu, idx_ref, b_ref):
    band = in_band(b_ref)
    ok = ~band
    mism_out = int((idx_gpu[ok] != idx_ref[ok]).sum())
    agree = float((idx_gpu == idx_ref).mean())
    return mism_out, agree, float(band.mean())

"""MI355X-native video-tokenizer round trip (encode -> FSQ -> token drop ->
decode) of arXiv 2602.03529, as hand-written CDNA4 HIP kernels behind the
C ABI in include/tok.h.  ``tok`` is the PyTorch binding (device memory and
streams only)."""
import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PACKAGE_DIR, "libtok.so")

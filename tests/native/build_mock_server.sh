#!/bin/bash
# Builds tests/native/libtok_serve_mock.so: the streaming server's source
# linked against host-only stand-ins of the HIP runtime and kernels (CPU tests).
set -e
HERE="$(cd "$(dirname "$0")" && pwd)"
ROOT="$(cd "$HERE/../.." && pwd)"
g++ -std=c++17 -O1 -g -fPIC -shared -D__HIP_PLATFORM_AMD__ -I/opt/rocm/include -I"$ROOT/include" \
  -x c++ "$ROOT/paper_2602_03529_amd/csrc/tok_serve.hip" -x c++ "$HERE/mock_runtime.cpp" \
  -o "$HERE/libtok_serve_mock.so" -lpthread

#!/bin/bash
# Builds and runs the two-stream concurrency micro-benchmark (needs an MI355X).
set -e
HERE=$(cd "$(dirname "$0")" && pwd)
/opt/rocm/bin/hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
    -o "$HERE/overlap_probe" "$HERE/overlap_probe.hip" 2>/dev/null
"$HERE/overlap_probe"

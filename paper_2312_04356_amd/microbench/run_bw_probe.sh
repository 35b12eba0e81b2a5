#!/bin/bash
# Builds and runs the HBM streaming micro-benchmark (needs an MI355X).
set -e
HERE=$(cd "$(dirname "$0")" && pwd)
/opt/rocm/bin/hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
    -o "$HERE/bw_probe" "$HERE/bw_probe.hip" 2>/dev/null
"$HERE/bw_probe"

#!/bin/bash
# Builds libpmr.so (gfx950) next to this script: every translation unit (one per FFT size)
# is compiled in parallel, then linked. Usage: build.sh [extra hipcc flags]
set -euo pipefail
here="$(cd "$(dirname "${BASH_SOURCE[0]}")" && pwd)"
src="$here/csrc"
out="$here/libpmr.so"
obj="$(mktemp -d "${TMPDIR:-/tmp}/pmr_build.XXXXXX")"
trap 'rm -rf "$obj"' EXIT
flags=(--offload-arch=gfx950 -O3 -std=c++17 -fPIC
       -Xclang -target-feature -Xclang -packed-fp32-ops
       -I"$here/../include" -I"$src")
jobs=${MAX_JOBS:-8}
[ "$jobs" -gt 16 ] && jobs=16
units=()
for n in 16 32 64 128 256 512; do units+=("fft_size.hip:-DPMR_FFT_SIZE=$n:fft_$n.o"); done
for f in fft.hip cic.hip sort.hip halo.hip halo2.hip recon.hip lpt2.hip pmr.cpp; do units+=("$f::${f%.*}.o"); done
pids=()
status=0
for u in "${units[@]}"; do
  IFS=: read -r file def o <<< "$u"
  while [ "$(jobs -rp | wc -l)" -ge "$jobs" ]; do sleep 0.2; done
  hipcc "${flags[@]}" $def "$@" -c "$src/$file" -o "$obj/$o" &
  pids+=($!)
done
for p in "${pids[@]}"; do wait "$p" || status=1; done
[ "$status" -eq 0 ] || { echo "build failed" >&2; exit 1; }
hipcc --offload-arch=gfx950 -shared -fPIC "$obj"/*.o -o "$out.tmp$$"
mv -f "$out.tmp$$" "$out"
echo "built $out"

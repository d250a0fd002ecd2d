// Staging of a batch of device query sets into tile CSR arrays: one pass
// over every piece's offsets (lengths, code spans and checks) with a single
// read-back, then one gather launch, instead of a synchronous read of every
// set's offsets and a copy per set.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "sd_host.h"

namespace sd {

namespace {

// chunks of at most stage_chunk() sequences, piece by piece
std::vector<StageChunk> make_chunks(const std::vector<StagePiece>& pieces) {
  std::vector<StageChunk> ch;
  const int64_t step = stage_chunk();
  for (size_t p = 0; p < pieces.size(); ++p)
    for (int64_t y = pieces[p].first; y < pieces[p].first + pieces[p].count; y += step)
      ch.push_back(StageChunk{(uint32_t)p, 0u, y,
                              std::min<int64_t>(step, pieces[p].first + pieces[p].count - y)});
  return ch;
}

template <typename T>
T* upload(Scratch& sc, const std::vector<T>& v, hipStream_t s) {
  T* d = sc.get<T>(v.size());
  if (!v.empty())
    hip_check(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s),
              "upload staging table");
  return d;
}

}  // namespace

void stage_spans(sd_ctx* c, Scratch& sc, const sd_seqs* sets, std::vector<BatchPiece>& pieces,
                 bool want_hist, hipStream_t s) {
  if (pieces.empty()) return;
  std::vector<StagePiece> tab(pieces.size());
  for (size_t p = 0; p < pieces.size(); ++p) {
    const sd_seqs& st = sets[pieces[p].set];
    if (!st.on_device) throw Error{SD_E_INVAL, "device staging takes device sets"};
    tab[p] = StagePiece{st.offsets, st.codes, pieces[p].first, pieces[p].count,
                        nullptr,    nullptr,  0,               0};
  }
  const std::vector<StageChunk> ch = make_chunks(tab);
  const StagePiece* dtab = upload(sc, tab, s);
  const StageChunk* dch = upload(sc, ch, s);
  const uint64_t nh = want_hist ? pieces.size() * STAGE_BINS : 0;
  // one block: the histogram, the spans and the error word
  uint8_t* blk = sc.get<uint8_t>(nh * 4 + pieces.size() * 16 + 16);
  uint32_t* hist = want_hist ? reinterpret_cast<uint32_t*>(blk) : nullptr;
  int64_t* spans = reinterpret_cast<int64_t*>(blk + nh * 4);
  uint32_t* err = reinterpret_cast<uint32_t*>(blk + nh * 4 + pieces.size() * 16);
  launch_fill_u32(reinterpret_cast<uint32_t*>(blk), 0,
                  (nh * 4 + pieces.size() * 16 + 16) / 4, s);
  launch_stage_spans(dtab, dch, (uint32_t)ch.size(), hist, spans, err, s);
  std::vector<uint8_t> h(nh * 4 + pieces.size() * 16 + 16);
  hip_check(hipMemcpyAsync(h.data(), blk, h.size(), hipMemcpyDeviceToHost, s), "read spans");
  hip_check(hipStreamSynchronize(s), "synchronise");
  uint32_t e;
  std::memcpy(&e, h.data() + nh * 4 + pieces.size() * 16, 4);
  raise_validation(e);
  for (size_t p = 0; p < pieces.size(); ++p) {
    std::memcpy(&pieces[p].lo, h.data() + nh * 4 + p * 16, 8);
    std::memcpy(&pieces[p].hi, h.data() + nh * 4 + p * 16 + 8, 8);
    if (want_hist) {
      std::memcpy(pieces[p].hist, h.data() + p * STAGE_BINS * 4, STAGE_BINS * 4);
      if (pieces[p].hist[0]) throw Error{SD_E_LENGTH, "a sequence length is outside [1, 24]"};
    }
  }
}

void stage_gather(sd_ctx* c, Scratch& sc, const sd_seqs* sets,
                  const std::vector<BatchPiece>& pieces, hipStream_t s) {
  (void)c;
  if (pieces.empty()) return;
  std::vector<StagePiece> tab(pieces.size());
  for (size_t p = 0; p < pieces.size(); ++p) {
    const BatchPiece& b = pieces[p];
    tab[p] = StagePiece{sets[b.set].offsets, sets[b.set].codes, b.first, b.count,
                        b.dst_offs,          b.dst_codes,       b.lo,    b.cbase};
  }
  const std::vector<StageChunk> ch = make_chunks(tab);
  const StagePiece* dtab = upload(sc, tab, s);
  const StageChunk* dch = upload(sc, ch, s);
  launch_stage_gather(dtab, dch, (uint32_t)ch.size(), s);
  // the tables are host vectors of this scope
  hip_check(hipStreamSynchronize(s), "synchronise");
}

}  // namespace sd

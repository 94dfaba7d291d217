// Index files (host code only): the versioned, checksummed container of an
// ann_index_desc documented in include/ann.h -- a 128-byte header, a table
// of sections with one CRC-32 each, then the arrays at 64-byte boundaries.
//
// The reader maps the file, checks everything it can on the host (header,
// table, sizes, checksums, then the checks of ann_index_create on the
// arrays) and only then touches a GPU.  The writer lays a description out in
// the same format.
#include <fcntl.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cstdio>
#include <cstring>
#include <vector>

#include "ann.h"
#include "internal.h"

using namespace ann;

namespace {

constexpr char kMagic[8] = {'A', 'N', 'N', 'I', 'N', 'D', 'E', 'X'};
constexpr uint32_t kVersion = 1;
constexpr size_t kHeaderBytes = 128;
constexpr size_t kEntryBytes = 32;
constexpr size_t kAlign = 64;
constexpr int kSections = 14;

enum Section {
  S_LEVELS = 1, S_ADJ0, S_UPPER_OFF, S_UPPER_ADJ, S_X_F32, S_X_F16, S_X_BF16, S_X_FP8,
  S_FP8_SCALE, S_PQ_CODEBOOK, S_PQ_CODES, S_SP_INDPTR, S_SP_IDS, S_SP_VALS
};

const char* section_name(int id) {
  static const char* names[] = {"?", "levels", "adj0", "upper_off", "upper_adj", "x_f32", "x_f16",
                                "x_bf16", "x_fp8", "fp8_scale", "pq_codebook", "pq_codes",
                                "sp_indptr", "sp_ids", "sp_vals"};
  return (id >= 1 && id <= kSections) ? names[id] : names[0];
}

// CRC-32 (IEEE 802.3, reflected polynomial 0xEDB88320), eight bytes per
// step with eight derived tables.
struct Crc32 {
  uint32_t t[8][256];
  Crc32() {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t c = i;
      for (int k = 0; k < 8; ++k) c = (c & 1u) ? (c >> 1) ^ 0xEDB88320u : c >> 1;
      t[0][i] = c;
    }
    for (uint32_t i = 0; i < 256; ++i)
      for (int s = 1; s < 8; ++s) t[s][i] = (t[s - 1][i] >> 8) ^ t[0][t[s - 1][i] & 0xFFu];
  }
  uint32_t operator()(const void* data, size_t len) const {
    const uint8_t* p = (const uint8_t*)data;
    uint32_t c = 0xFFFFFFFFu;
    while (len >= 8) {
      uint32_t lo, hi;
      std::memcpy(&lo, p, 4);
      std::memcpy(&hi, p + 4, 4);
      lo ^= c;
      c = t[7][lo & 0xFF] ^ t[6][(lo >> 8) & 0xFF] ^ t[5][(lo >> 16) & 0xFF] ^ t[4][lo >> 24] ^
          t[3][hi & 0xFF] ^ t[2][(hi >> 8) & 0xFF] ^ t[1][(hi >> 16) & 0xFF] ^ t[0][hi >> 24];
      p += 8;
      len -= 8;
    }
    while (len--) c = (c >> 8) ^ t[0][(c ^ *p++) & 0xFFu];
    return c ^ 0xFFFFFFFFu;
  }
};

const Crc32& crc32() {
  static const Crc32 table;
  return table;
}

struct Header {
  uint32_t sections;
  int64_t n;
  int32_t d, metric, M, M0, max_level, entry_point;
  int64_t n_upper_lists;
  int32_t pq_m, pq_ksub;
  int64_t nnz;
};

template <class T>
T get(const uint8_t* p) {
  T v;
  std::memcpy(&v, p, sizeof v);
  return v;
}

template <class T>
void put(uint8_t* p, T v) {
  std::memcpy(p, &v, sizeof v);
}

// The size every section must have under the header's fields (0: the header
// rules the section out).
uint64_t expected_size(const Header& h, int id) {
  const uint64_t n = (uint64_t)h.n, d = (uint64_t)h.d;
  switch (id) {
    case S_LEVELS: return n;
    case S_ADJ0: return n * h.M0 * 4;
    case S_UPPER_OFF: return n * 4;
    case S_UPPER_ADJ: return (uint64_t)h.n_upper_lists * h.M * 4;
    case S_X_F32: return n * d * 4;
    case S_X_F16: case S_X_BF16: return n * d * 2;
    case S_X_FP8: return n * d;
    case S_FP8_SCALE: return n * 4;
    case S_PQ_CODEBOOK: return h.pq_m > 0 ? 256 * d * 4 : 0;
    case S_PQ_CODES: return n * (uint64_t)h.pq_m;
    case S_SP_INDPTR: return h.nnz > 0 ? (n + 1) * 8 : 0;
    case S_SP_IDS: return (uint64_t)h.nnz * 2;
    case S_SP_VALS: return (uint64_t)h.nnz * 4;
  }
  return 0;
}

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Offset of the first section: header, table and its CRC, aligned.
uint64_t table_end(uint32_t sections) {
  return align_up(kHeaderBytes + (uint64_t)sections * kEntryBytes + 4);
}

// A read-only mapping of a whole file.
struct Mapping {
  int fd = -1;
  const uint8_t* base = nullptr;
  size_t size = 0;
  ~Mapping() {
    if (base && size) munmap((void*)base, size);
    if (fd >= 0) close(fd);
  }
};

int map_file(const char* path, Mapping& m) {
  m.fd = open(path, O_RDONLY);
  if (m.fd < 0) return fail(ANN_EINVAL, "cannot open index file %s", path);
  struct stat st;
  if (fstat(m.fd, &st) != 0) return fail(ANN_EINVAL, "cannot stat index file %s", path);
  m.size = (size_t)st.st_size;
  if (m.size < kHeaderBytes)
    return fail(ANN_EFORMAT, "index file of %zu bytes is shorter than its header", m.size);
  void* p = mmap(nullptr, m.size, PROT_READ, MAP_PRIVATE, m.fd, 0);
  if (p == MAP_FAILED) {
    m.size = 0;
    return fail(ANN_EINVAL, "cannot map index file %s", path);
  }
  m.base = (const uint8_t*)p;
  return ANN_OK;
}

// Checks the header, the table and every section of a mapped file and
// points the description's arrays at the sections.
int parse(const Mapping& m, ann_index_desc* D, Header* hout) {
  const uint8_t* b = m.base;
  if (std::memcmp(b, kMagic, 8) != 0) return fail(ANN_EFORMAT, "not an index file (magic)");
  const uint32_t version = get<uint32_t>(b + 8);
  if (version != kVersion)
    return fail(ANN_EFORMAT, "index file version %u, this library reads version %u", version, kVersion);
  if (crc32()(b, 124) != get<uint32_t>(b + 124)) return fail(ANN_EFORMAT, "header checksum mismatch");
  Header h;
  h.sections = get<uint32_t>(b + 12);
  h.n = get<int64_t>(b + 16);
  h.d = get<int32_t>(b + 24);
  h.metric = get<int32_t>(b + 28);
  h.M = get<int32_t>(b + 32);
  h.M0 = get<int32_t>(b + 36);
  h.max_level = get<int32_t>(b + 40);
  h.entry_point = get<int32_t>(b + 44);
  h.n_upper_lists = get<int64_t>(b + 48);
  h.pq_m = get<int32_t>(b + 56);
  h.pq_ksub = get<int32_t>(b + 60);
  h.nnz = get<int64_t>(b + 64);
  for (int i = 72; i < 124; ++i)
    if (b[i] != 0) return fail(ANN_EFORMAT, "reserved header byte %d is not zero", i);
  if (h.sections < 1 || h.sections > kSections)
    return fail(ANN_EFORMAT, "section count %u outside [1, %d]", h.sections, kSections);
  if (h.n < 1 || h.n > INT32_MAX - 1) return fail(ANN_EFORMAT, "n %lld outside [1, 2^31 - 2]", (long long)h.n);
  if (h.d < 1 || h.d > (1 << 20)) return fail(ANN_EFORMAT, "d %d outside [1, 2^20]", h.d);
  if (h.M < 1 || h.M > 64 || h.M0 < 1 || h.M0 > 64)
    return fail(ANN_EFORMAT, "need 1 <= M <= 64 and 1 <= M0 <= 64 (M=%d M0=%d)", h.M, h.M0);
  if (h.n_upper_lists < 0 || h.n_upper_lists > (int64_t)h.n * 64)
    return fail(ANN_EFORMAT, "n_upper_lists %lld out of range", (long long)h.n_upper_lists);
  if (h.pq_m < 0 || h.pq_m > 64 || (h.pq_m > 0 && (h.pq_ksub != 256 || h.d % h.pq_m != 0)) ||
      (h.pq_m == 0 && h.pq_ksub != 0))
    return fail(ANN_EFORMAT, "PQ fields pq_m=%d pq_ksub=%d invalid for d=%d", h.pq_m, h.pq_ksub, h.d);
  if (h.nnz < 0 || h.nnz > ((int64_t)1 << 40)) return fail(ANN_EFORMAT, "nnz %lld out of range", (long long)h.nnz);
  const uint64_t tab = kHeaderBytes + (uint64_t)h.sections * kEntryBytes;
  if (m.size < tab + 4) return fail(ANN_EFORMAT, "index file truncated inside its section table");
  if (crc32()(b + kHeaderBytes, tab - kHeaderBytes) != get<uint32_t>(b + tab))
    return fail(ANN_EFORMAT, "section table checksum mismatch");
  std::memset(D, 0, sizeof *D);
  D->n = h.n; D->d = h.d; D->metric = h.metric; D->M = h.M; D->M0 = h.M0;
  D->max_level = h.max_level; D->entry_point = h.entry_point; D->n_upper_lists = h.n_upper_lists;
  const void* at[kSections + 1] = {};
  int prev = 0;
  uint64_t end = tab + 4;   // the table's CRC ends here
  for (uint32_t i = 0; i < h.sections; ++i) {
    const uint8_t* e = b + kHeaderBytes + (size_t)i * kEntryBytes;
    const int id = (int)get<uint32_t>(e);
    const uint32_t crc = get<uint32_t>(e + 4);
    const uint64_t off = get<uint64_t>(e + 8), size = get<uint64_t>(e + 16);
    if (id < 1 || id > kSections) return fail(ANN_EFORMAT, "unknown section id %d", id);
    if (id <= prev) return fail(ANN_EFORMAT, "section %s out of order or repeated", section_name(id));
    if (get<uint64_t>(e + 24) != 0) return fail(ANN_EFORMAT, "section %s: reserved field not zero", section_name(id));
    // each section starts at the first 64-byte boundary after what precedes
    // it, with zero bytes in between
    if (off != align_up(end))
      return fail(ANN_EFORMAT, "section %s at offset %llu: misaligned or misplaced (expected %llu)", section_name(id),
                  (unsigned long long)off, (unsigned long long)align_up(end));
    const uint64_t want = expected_size(h, id);
    if (want == 0 || size != want)
      return fail(ANN_EFORMAT, "section %s has %llu bytes, the header implies %llu", section_name(id),
                  (unsigned long long)size, (unsigned long long)want);
    if (off > m.size || size > m.size - off)
      return fail(ANN_EFORMAT, "index file truncated inside section %s", section_name(id));
    for (uint64_t z = end; z < off; ++z)
      if (b[z] != 0)
        return fail(ANN_EFORMAT, "nonzero padding byte at offset %llu before section %s",
                    (unsigned long long)z, section_name(id));
    if (crc32()(b + off, size) != crc) return fail(ANN_EFORMAT, "section %s checksum mismatch", section_name(id));
    at[id] = b + off;
    prev = id;
    end = off + size;
  }
  if (end != m.size) return fail(ANN_EFORMAT, "%llu bytes after the last section", (unsigned long long)(m.size - end));
  for (int id : {S_LEVELS, S_ADJ0, S_UPPER_OFF})
    if (!at[id]) return fail(ANN_EFORMAT, "required section %s missing", section_name(id));
  if ((h.n_upper_lists > 0) != (at[S_UPPER_ADJ] != nullptr))
    return fail(ANN_EFORMAT, "upper_adj present iff n_upper_lists > 0");
  if ((at[S_X_FP8] != nullptr) != (at[S_FP8_SCALE] != nullptr))
    return fail(ANN_EFORMAT, "x_fp8 and fp8_scale go together");
  if ((h.pq_m > 0) != (at[S_PQ_CODEBOOK] != nullptr) || (h.pq_m > 0) != (at[S_PQ_CODES] != nullptr))
    return fail(ANN_EFORMAT, "pq_codebook and pq_codes present iff pq_m > 0");
  const bool sp = h.nnz > 0;
  if (sp != (at[S_SP_INDPTR] != nullptr) || sp != (at[S_SP_IDS] != nullptr) || sp != (at[S_SP_VALS] != nullptr))
    return fail(ANN_EFORMAT, "sp_indptr, sp_ids and sp_vals present iff nnz > 0");
  if (sp && get<int64_t>((const uint8_t*)at[S_SP_INDPTR] + 8 * (size_t)h.n) != h.nnz)
    return fail(ANN_EFORMAT, "sp_indptr[n] differs from the header's nnz");
  D->levels = (const uint8_t*)at[S_LEVELS];
  D->adj0 = (const int32_t*)at[S_ADJ0];
  D->upper_off = (const int32_t*)at[S_UPPER_OFF];
  D->upper_adj = (const int32_t*)at[S_UPPER_ADJ];
  D->x_f32 = (const float*)at[S_X_F32];
  D->x_f16 = (const uint16_t*)at[S_X_F16];
  D->x_bf16 = (const uint16_t*)at[S_X_BF16];
  D->x_fp8 = (const uint8_t*)at[S_X_FP8];
  D->fp8_scale = (const float*)at[S_FP8_SCALE];
  D->pq_m = h.pq_m;
  D->pq_ksub = h.pq_ksub;
  D->pq_codebook = (const float*)at[S_PQ_CODEBOOK];
  D->pq_codes = (const uint8_t*)at[S_PQ_CODES];
  D->sp_indptr = (const int64_t*)at[S_SP_INDPTR];
  D->sp_ids = (const uint16_t*)at[S_SP_IDS];
  D->sp_vals = (const float*)at[S_SP_VALS];
  // everything ann_index_create checks; its ANN_EINVAL cases are format
  // errors in a file
  const int rc = check_desc(D);
  if (rc == ANN_EINVAL) return ANN_EFORMAT;
  if (rc) return rc;
  *hout = h;
  return ANN_OK;
}

void fill_info(const Header& h, const ann_index_desc& D, const Mapping& m, ann_info* out) {
  std::memset(out, 0, sizeof *out);
  out->n = h.n; out->d = h.d; out->metric = h.metric; out->M = h.M; out->M0 = h.M0;
  out->max_level = h.max_level; out->entry_point = h.entry_point;
  if (D.x_f32) out->modes |= 1 << ANN_MODE_F32;
  if (D.x_f16) out->modes |= 1 << ANN_MODE_F16;
  if (D.x_bf16) out->modes |= 1 << ANN_MODE_BF16;
  if (D.x_fp8) out->modes |= 1 << ANN_MODE_FP8;
  if (D.pq_codes) out->modes |= 1 << ANN_MODE_PQ;
  if (D.sp_indptr) out->modes |= 1 << ANN_MODE_SPARSE;
  out->device = -1;
  out->device_bytes = (int64_t)(m.size - table_end(h.sections));
}

}  // namespace

extern "C" {

int ann_index_file_info(const char* path, ann_info* out) {
  if (!path || !out) return fail(ANN_EINVAL, "NULL argument");
  Mapping m;
  int rc = map_file(path, m);
  if (rc) return rc;
  ann_index_desc D;
  Header h;
  if ((rc = parse(m, &D, &h))) return rc;
  fill_info(h, D, m, out);
  return ANN_OK;
}

int ann_index_load(const char* path, int device, ann_index** out) {
  if (!path || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  Mapping m;
  int rc = map_file(path, m);
  if (rc) return rc;
  ann_index_desc D;
  Header h;
  if ((rc = parse(m, &D, &h))) return rc;
  return ann_index_create(&D, device, out);
}

int ann_index_save(const ann_index_desc* D, const char* path) {
  if (!D || !path) return fail(ANN_EINVAL, "NULL argument");
  int rc = check_desc(D);
  if (rc) return rc;
  Header h;
  h.n = D->n; h.d = D->d; h.metric = D->metric; h.M = D->M; h.M0 = D->M0;
  h.max_level = D->max_level; h.entry_point = D->entry_point; h.n_upper_lists = D->n_upper_lists;
  h.pq_m = D->pq_codes ? D->pq_m : 0;
  h.pq_ksub = D->pq_codes ? 256 : 0;
  h.nnz = D->sp_indptr ? D->sp_indptr[D->n] : 0;
  const void* data[kSections + 1] = {nullptr, D->levels, D->adj0, D->upper_off,
                                     D->n_upper_lists > 0 ? D->upper_adj : nullptr, D->x_f32,
                                     D->x_f16, D->x_bf16, D->x_fp8, D->x_fp8 ? D->fp8_scale : nullptr,
                                     D->pq_codes ? D->pq_codebook : nullptr, D->pq_codes,
                                     h.nnz > 0 ? D->sp_indptr : nullptr, h.nnz > 0 ? D->sp_ids : nullptr,
                                     h.nnz > 0 ? D->sp_vals : nullptr};
  std::vector<int> ids;
  for (int id = 1; id <= kSections; ++id)
    if (data[id]) ids.push_back(id);
  h.sections = (uint32_t)ids.size();
  std::vector<uint8_t> head(table_end(h.sections), 0);
  std::memcpy(head.data(), kMagic, 8);
  put<uint32_t>(&head[8], kVersion);
  put<uint32_t>(&head[12], h.sections);
  put<int64_t>(&head[16], h.n);
  put<int32_t>(&head[24], h.d);
  put<int32_t>(&head[28], h.metric);
  put<int32_t>(&head[32], h.M);
  put<int32_t>(&head[36], h.M0);
  put<int32_t>(&head[40], h.max_level);
  put<int32_t>(&head[44], h.entry_point);
  put<int64_t>(&head[48], h.n_upper_lists);
  put<int32_t>(&head[56], h.pq_m);
  put<int32_t>(&head[60], h.pq_ksub);
  put<int64_t>(&head[64], h.nnz);
  put<uint32_t>(&head[124], crc32()(head.data(), 124));
  uint64_t off = head.size();
  std::vector<uint64_t> offs;
  for (size_t i = 0; i < ids.size(); ++i) {
    const int id = ids[i];
    const uint64_t size = expected_size(h, id);
    uint8_t* e = &head[kHeaderBytes + i * kEntryBytes];
    put<uint32_t>(e, (uint32_t)id);
    put<uint32_t>(e + 4, crc32()(data[id], size));
    put<uint64_t>(e + 8, off);
    put<uint64_t>(e + 16, size);
    offs.push_back(off);
    off = align_up(off + size);
  }
  const size_t tab = kHeaderBytes + ids.size() * kEntryBytes;
  put<uint32_t>(&head[tab], crc32()(&head[kHeaderBytes], tab - kHeaderBytes));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(ANN_EINVAL, "cannot write index file %s", path);
  bool ok = std::fwrite(head.data(), 1, head.size(), f) == head.size();
  uint64_t pos = head.size();
  static const uint8_t zeros[kAlign] = {};
  for (size_t i = 0; ok && i < ids.size(); ++i) {
    if (offs[i] > pos) ok = std::fwrite(zeros, 1, offs[i] - pos, f) == offs[i] - pos;
    const uint64_t size = expected_size(h, ids[i]);
    ok = ok && std::fwrite(data[ids[i]], 1, size, f) == size;
    pos = offs[i] + size;
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(ANN_EINVAL, "writing index file %s failed", path);
  return ANN_OK;
}

}  // extern "C"
